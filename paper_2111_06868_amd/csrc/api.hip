// extern "C" entry points declared in include/sv.h: states, gates, fusion,
// circuits, reductions, adjoint gradients and timing.
#include <hip/hip_runtime.h>

#include <atomic>
#include <fstream>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "runtime.h"

namespace sv {
const char *last_error_cstr();
int stats_enable(int on);
int stats_reset();
int stats_query(int cls, int64_t *launches, double *total_ms);
}  // namespace sv

using namespace sv;

namespace {

constexpr int kVersion = 1;

size_t amp_bytes(int dtype) { return dtype == SV_C64 ? 8 : 16; }

int check_state(const sv_state *s)
{
    if (!s) return fail(SV_ERR_ARG, "NULL state handle");
    return SV_OK;
}

int select_device(const sv_state *s)
{
    SV_HIP(hipSetDevice(s->device));
    return SV_OK;
}

// Make `to` wait for the work already enqueued on `from`.
int stream_after(hipStream_t to, hipStream_t from)
{
    if (to == from) return SV_OK;
    hipEvent_t e;
    SV_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    SV_HIP(hipEventRecord(e, from));
    SV_HIP(hipStreamWaitEvent(to, e, 0));
    SV_HIP(hipEventDestroy(e));
    return SV_OK;
}

int check_precision(const sv_state *s, int precision)
{
    if (precision < SV_PREC_FP32 || precision > SV_PREC_SPLIT_BF16X3) return fail(SV_ERR_ARG, "unknown precision %d", precision);
    if ((s->dtype == SV_C128) != (precision == SV_PREC_FP64))
        return fail(SV_ERR_ARG, "precision %d does not match the state's amplitude type", precision);
    return SV_OK;
}

int validate_gates(const sv_gate *g, int G, int n)
{
    if (G < 0) return fail(SV_ERR_ARG, "negative gate count");
    if (G > 0 && !g) return fail(SV_ERR_ARG, "NULL gate array");
    for (int i = 0; i < G; ++i) {
        int rc = check_gate_shape(g[i]);
        if (!rc) rc = check_gate_qubits(g[i], n);
        if (rc) {
            std::string msg = std::string("gate ") + std::to_string(i) + ": " + last_error_cstr();
            return fail(rc, "%s", msg.c_str());
        }
    }
    return SV_OK;
}

// Upload `bytes` staged bytes and enqueue `launches`; the arena and staging
// buffers are reused only after the previous user of the arena finished.
int run_launches(sv_state *s, std::vector<Launch> &launches, bool use_graph)
{
    SV_HIP(hipEventSynchronize(s->arena_free));
    const size_t bytes = pack_operands(launches, s->dtype, s->stage);
    if (bytes == size_t(-1)) return fail(SV_ERR_HIP, "pinned staging allocation failed");
    if (bytes) {
        SV_HIP(s->arena.ensure(bytes));
        SV_HIP(hipMemcpyAsync(s->arena.p, s->stage.p, bytes, hipMemcpyHostToDevice, s->stream));
    }
    if (!use_graph) {
        int rc = enqueue(launches, s->dtype, s->buf, s->n, s->arena.p, s->stream);
        SV_HIP(hipEventRecord(s->arena_free, s->stream));
        return rc;
    }
    // Capture the launches, then reuse the state's instantiated graph when the
    // new one has the same topology (hipGraphExecUpdate takes the new kernel
    // arguments: matrices, operand addresses), else instantiate anew.  The
    // previous launch of that graph has finished: arena_free was synchronised.
    if (!s->capture_stream) SV_HIP(hipStreamCreateWithFlags(&s->capture_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    SV_HIP(hipStreamBeginCapture(s->capture_stream, hipStreamCaptureModeThreadLocal));
    timing_suspend(true);
    int rc = enqueue(launches, s->dtype, s->buf, s->n, s->arena.p, s->capture_stream);
    timing_suspend(false);
    hipError_t e = hipStreamEndCapture(s->capture_stream, &graph);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(SV_ERR_HIP, "graph capture: %s", hipGetErrorString(e));
    bool updated = false;
    if (s->graph_exec) {
        hipGraphNode_t bad = nullptr;
        hipGraphExecUpdateResult res = hipGraphExecUpdateError;
        updated = hipGraphExecUpdate(s->graph_exec, graph, &bad, &res) == hipSuccess && res == hipGraphExecUpdateSuccess;
        if (!updated) {
            (void)hipGetLastError();  // a refused update is not an error of this call
            (void)hipGraphExecDestroy(s->graph_exec);
            s->graph_exec = nullptr;
        }
    }
    if (!updated) e = hipGraphInstantiate(&s->graph_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e == hipSuccess) e = hipGraphLaunch(s->graph_exec, s->stream);
    if (e == hipSuccess) e = hipEventRecord(s->arena_free, s->stream);
    if (e != hipSuccess) {
        if (s->graph_exec) (void)hipGraphExecDestroy(s->graph_exec);
        s->graph_exec = nullptr;
        return fail(SV_ERR_HIP, "graph launch: %s", hipGetErrorString(e));
    }
    ++s->graph_launches;
    if (updated) ++s->graph_updates;
    return SV_OK;
}

void blocks_to_launches(const std::vector<Block> &blocks, const sv_state *s, int precision, int rule,
                        std::vector<Launch> &out)
{
    if (rule == SV_RULE_TILED && s->dtype == SV_C64 && precision != SV_PREC_FP64) {
        group_tile_passes(blocks, s->n, precision, out);
        return;
    }
    out.clear();
    out.reserve(blocks.size());
    for (const auto &b : blocks) {
        Launch L;
        L.k = b.k;
        std::copy(b.q, b.q + SV_MAX_K, L.q);
        L.path = choose_path(s->dtype, precision, b.k, b.q, s->n);
        L.m = b.m;
        out.push_back(std::move(L));
    }
}

int choose_plan_uncached(const sv_gate *g, int G, int n, int dtype, int precision, int rule, int max_k, bool found,
                         const CostTable &cost, int kmin, int kcap, int *out_rule, int *out_k);

// Resolve (rule, max_k) requests: max_k = -1 picks k by the cost table;
// SV_RULE_AUTO also picks between the enhanced and the tiled plan.  Candidate
// plans are priced on block positions only (no matrices are formed).
int choose_plan(const sv_gate *g, int G, int n, int dtype, int precision, int rule, int max_k, int *out_rule,
                int *out_k)
{
    bool found = false;
    const CostTable cost = lookup_costs(n, precision, &found);
    int kmin = 1;
    for (int i = 0; i < G; ++i) kmin = std::max(kmin, g[i].k);
    const int kcap = max_k > 0 ? max_k : SV_MAX_K;
    if (max_k > 0 && rule != SV_RULE_AUTO) {
        *out_rule = rule;
        *out_k = max_k;
        return SV_OK;
    }
    // The choice depends on the gates' positions and the cost table only, so
    // it is remembered per circuit structure (a circuit re-run with new
    // angles is not re-priced).  A stale or colliding entry can only name
    // another valid (rule, k), and one below the widest gate is recomputed.
    uint64_t key = 1469598103934665603ull;
    auto mix = [&key](uint64_t v) { key = (key ^ v) * 1099511628211ull; };
    mix(uint64_t(n));
    mix(uint64_t(dtype));
    mix(uint64_t(precision));
    mix(uint64_t(rule));
    mix(uint64_t(max_k + 8));
    mix(cost_version());
    mix(uint64_t(tile_union_limit()));
    mix(uint64_t(tile_pass_bits()) | uint64_t(tile_pass_capacity(precision)) << 8);
    mix(uint64_t(G));
    for (int i = 0; i < G; ++i) {
        mix(uint64_t(g[i].kind) | uint64_t(g[i].k) << 8);
        for (int j = 0; j < g[i].k; ++j) mix(uint64_t(g[i].q[j]));
    }
    static std::mutex memo_mu;
    static std::unordered_map<uint64_t, std::pair<int, int>> memo;
    {
        std::lock_guard<std::mutex> lk(memo_mu);
        auto it = memo.find(key);
        if (it != memo.end() && it->second.second >= kmin) {
            *out_rule = it->second.first;
            *out_k = it->second.second;
            return SV_OK;
        }
    }
    const int rc = choose_plan_uncached(g, G, n, dtype, precision, rule, max_k, found, cost, kmin, kcap, out_rule,
                                        out_k);
    if (!rc) {
        std::lock_guard<std::mutex> lk(memo_mu);
        if (memo.size() > 4096) memo.clear();
        memo[key] = {*out_rule, *out_k};
    }
    return rc;
}

int choose_plan_uncached(const sv_gate *g, int G, int n, int dtype, int precision, int rule, int max_k, bool found,
                         const CostTable &cost, int kmin, int kcap, int *out_rule, int *out_k)
{
    std::vector<int> rules;
    if (rule == SV_RULE_AUTO) {
        rules.push_back(SV_RULE_ENHANCED);
        if (dtype == SV_C64 && precision != SV_PREC_FP64 && n >= dev::kMinTileQubits) rules.push_back(SV_RULE_TILED);
    } else {
        rules.push_back(rule == SV_RULE_NONE ? SV_RULE_PAPER : rule);
    }
    double best = 1e300;
    int best_rule = rules[0], best_k = std::min(kmin, kcap);
    for (int r : rules) {
        const int khi = std::min(kcap, r == SV_RULE_TILED ? 4 : SV_MAX_K);
        for (int k = kmin; k <= khi; ++k) {
            if (!found && k == SV_MAX_K) break;  // untuned: stay below the MFMA-bound size
            std::vector<Block> blocks;
            if (int rc = fuse_gates(g, G, n, k, r, cost, blocks, false, precision)) return rc;
            const double c = r == SV_RULE_TILED ? tiled_plan_cost(blocks, n, cost) : plan_cost(blocks, cost);
            if (c < best - 1e-12) {
                best = c;
                best_rule = r;
                best_k = k;
            }
        }
    }
    *out_rule = rule == SV_RULE_NONE ? SV_RULE_NONE : best_rule;
    *out_k = best_k;
    return SV_OK;
}

int pauli_tables(sv_state *s, const sv_pauli_sum *H, dev::PauliDev &P);

}  // namespace

// ============================================================== misc
extern "C" const char *sv_last_error(void) { return last_error_cstr(); }
extern "C" int sv_version(void) { return kVersion; }

// ============================================================== states
extern "C" int sv_alloc(int n, int dtype, void *dev_buf, size_t bytes, void *hip_stream, sv_state **out)
{
    clear_error();
    if (!out) return fail(SV_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (dtype != SV_C64 && dtype != SV_C128) return fail(SV_ERR_ARG, "unknown amplitude type %d", dtype);
    const int nmax = dtype == SV_C64 ? SV_MAX_QUBITS_C64 : SV_MAX_QUBITS_C128;
    if (n < 1 || n > nmax) return fail(SV_ERR_ARG, "n = %d outside 1..%d", n, nmax);
    const size_t need = (size_t(1) << n) * amp_bytes(dtype);
    if (dev_buf) {
        if (bytes < need) return fail(SV_ERR_SIZE, "buffer of %zu bytes < %zu needed for %d qubits", bytes, need, n);
        if (reinterpret_cast<uintptr_t>(dev_buf) % 256) return fail(SV_ERR_ARG, "device buffer not 256-byte aligned");
    }
    sv_state *s = new sv_state;
    s->n = n;
    s->dtype = dtype;
    s->stream = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->arena_free, hipEventDisableTiming);
    if (e == hipSuccess && !dev_buf) {
        e = hipMalloc(&s->buf, need);
        s->owns = e == hipSuccess;
        s->bytes = need;
    } else {
        s->buf = dev_buf;
        s->bytes = bytes;
    }
    if (e == hipSuccess) e = s->red.ensure(sizeof(double) * (2 * dev::kRedBlocks + 64));
    if (e == hipSuccess) e = s->red_host.ensure(sizeof(double) * 64);
    if (e == hipSuccess) e = dev::launch_fill_basis(dtype, s->buf, n, 0, s->stream);
    if (e != hipSuccess) {
        int rc = fail(SV_ERR_HIP, "sv_alloc: %s", hipGetErrorString(e));
        sv_free(s);
        return rc;
    }
    // the first state of the process installs a saved tuning cache, if any
    static std::once_flag cache_once;
    std::call_once(cache_once, [&] {
        const char *path = std::getenv("SV_TUNE_CACHE");
        if (path && *path && std::ifstream(path).good()) (void)load_tuning(path, s->device, nullptr);
        clear_error();
    });
    *out = s;
    return SV_OK;
}

extern "C" int sv_free(sv_state *s)
{
    if (!s) return SV_OK;
    (void)hipSetDevice(s->device);
    (void)hipStreamSynchronize(s->stream);
    if (s->owns && s->buf) (void)hipFree(s->buf);
    if (s->graph_exec) (void)hipGraphExecDestroy(s->graph_exec);
    if (s->capture_stream) (void)hipStreamDestroy(s->capture_stream);
    if (s->arena_free) (void)hipEventDestroy(s->arena_free);
    delete s;
    return SV_OK;
}

extern "C" int sv_info(const sv_state *s, int *n, int *dtype, void **dev_ptr)
{
    clear_error();
    if (int rc = check_state(s)) return rc;
    if (n) *n = s->n;
    if (dtype) *dtype = s->dtype;
    if (dev_ptr) *dev_ptr = s->buf;
    return SV_OK;
}

extern "C" int sv_set_product(sv_state *s, const char *tokens)
{
    clear_error();
    if (int rc = check_state(s)) return rc;
    if (!tokens) return fail(SV_ERR_ARG, "NULL tokens");
    const size_t len = std::strlen(tokens);
    if (len != 1 && len != size_t(s->n))
        return fail(SV_ERR_ARG, "initial state needs 1 or %d tokens, got %zu", s->n, len);
    double amps[4 * SV_MAX_QUBITS_C64];
    const double r = 0.70710678118654752440;
    for (int j = 0; j < s->n; ++j) {
        const char c = len == 1 ? tokens[0] : tokens[j];
        const int p = s->n - 1 - j;  // token j describes position n-1-j
        double *a = amps + 4 * p;
        switch (c) {
        case '0': a[0] = 1; a[1] = 0; a[2] = 0; a[3] = 0; break;
        case '1': a[0] = 0; a[1] = 0; a[2] = 1; a[3] = 0; break;
        case '+': a[0] = r; a[1] = 0; a[2] = r; a[3] = 0; break;
        case '-': a[0] = r; a[1] = 0; a[2] = -r; a[3] = 0; break;
        default: return fail(SV_ERR_ARG, "initial-state token '%c' is not one of 0 1 + -", c);
        }
    }
    if (int rc = select_device(s)) return rc;
    SV_HIP(dev::launch_product(s->dtype, s->buf, s->n, amps, s->stream));
    return SV_OK;
}

extern "C" int sv_set_basis(sv_state *s, uint64_t index)
{
    clear_error();
    if (int rc = check_state(s)) return rc;
    if (index >> s->n) return fail(SV_ERR_ARG, "basis index %llu >= 2^%d", (unsigned long long)index, s->n);
    if (int rc = select_device(s)) return rc;
    SV_HIP(dev::launch_fill_basis(s->dtype, s->buf, s->n, index, s->stream));
    return SV_OK;
}

extern "C" int sv_read(sv_state *s, uint64_t first, uint64_t count, void *host)
{
    clear_error();
    if (int rc = check_state(s)) return rc;
    const uint64_t N = uint64_t(1) << s->n;
    if (first > N || count > N - first) return fail(SV_ERR_ARG, "range [%llu, +%llu) outside the state", (unsigned long long)first, (unsigned long long)count);
    if (count && !host) return fail(SV_ERR_ARG, "NULL host buffer");
    if (int rc = select_device(s)) return rc;
    const size_t ab = amp_bytes(s->dtype);
    if (count) SV_HIP(hipMemcpyAsync(host, static_cast<char *>(s->buf) + first * ab, count * ab, hipMemcpyDeviceToHost, s->stream));
    SV_HIP(hipStreamSynchronize(s->stream));
    return SV_OK;
}

extern "C" int sv_write(sv_state *s, uint64_t first, uint64_t count, const void *host)
{
    clear_error();
    if (int rc = check_state(s)) return rc;
    const uint64_t N = uint64_t(1) << s->n;
    if (first > N || count > N - first) return fail(SV_ERR_ARG, "range outside the state");
    if (count && !host) return fail(SV_ERR_ARG, "NULL host buffer");
    if (int rc = select_device(s)) return rc;
    const size_t ab = amp_bytes(s->dtype);
    if (count) SV_HIP(hipMemcpyAsync(static_cast<char *>(s->buf) + first * ab, host, count * ab, hipMemcpyHostToDevice, s->stream));
    SV_HIP(hipStreamSynchronize(s->stream));
    return SV_OK;
}

extern "C" int sv_copy(sv_state *dst, sv_state *src)
{
    clear_error();
    if (!dst || !src) return fail(SV_ERR_ARG, "NULL state handle");
    if (dst->n != src->n) return fail(SV_ERR_ARG, "qubit counts differ (%d vs %d)", dst->n, src->n);
    if (int rc = select_device(dst)) return rc;
    if (int rc = stream_after(dst->stream, src->stream)) return rc;
    SV_HIP(dev::launch_convert(src->dtype, src->buf, dst->dtype, dst->buf, uint64_t(1) << dst->n, dst->stream));
    return SV_OK;
}

extern "C" int sv_synchronize(sv_state *s)
{
    clear_error();
    if (int rc = check_state(s)) return rc;
    if (int rc = select_device(s)) return rc;
    SV_HIP(hipStreamSynchronize(s->stream));
    return SV_OK;
}

// ============================================================== gates
extern "C" int sv_gate_matrix(const sv_gate *g, double *out)
{
    clear_error();
    if (!g || !out) return fail(SV_ERR_ARG, "NULL argument");
    std::vector<cd> m;
    if (int rc = gate_matrix_abi(*g, m)) return rc;
    for (size_t i = 0; i < m.size(); ++i) {
        out[2 * i] = m[i].real();
        out[2 * i + 1] = m[i].imag();
    }
    return SV_OK;
}

namespace {
int apply_gate_impl(sv_state *s, const sv_gate *g);
}

extern "C" int sv_apply_gate(sv_state *s, const sv_gate *g)
{
    clear_error();
    if (int rc = check_state(s)) return rc;
    if (int rc = validate_gates(g, 1, s->n)) return rc;
    return apply_gate_impl(s, g);
}

namespace {
int apply_gate_impl(sv_state *s, const sv_gate *g)
{
    Launch L;
    L.k = g->k;
    int sq[SV_MAX_K];
    if (int rc = gate_matrix_canonical(*g, L.m, sq)) return rc;
    std::fill(L.q, L.q + SV_MAX_K, 0);
    std::copy(sq, sq + g->k, L.q);
    const int prec = s->dtype == SV_C64 ? SV_PREC_FP32 : SV_PREC_FP64;
    L.path = choose_path(s->dtype, prec, L.k, L.q, s->n);
    std::vector<Launch> v;
    v.push_back(std::move(L));
    if (int rc = select_device(s)) return rc;
    return run_launches(s, v, false);
}
}  // namespace

// ============================================================== fusion
namespace {

// precision < 0: FP32 cost tables, tile passes sized for operands of any precision
int fuse_plan(const sv_gate *g, int G, int n, int max_k, int rule, int precision, sv_plan **out)
{
    if (!out) return fail(SV_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > SV_MAX_QUBITS_C64) return fail(SV_ERR_ARG, "n = %d outside 1..%d", n, SV_MAX_QUBITS_C64);
    if (precision < -1 || precision > SV_PREC_SPLIT_BF16X3) return fail(SV_ERR_ARG, "precision %d", precision);
    if (int rc = validate_gates(g, G, n)) return rc;
    if (rule < SV_RULE_PAPER || rule > SV_RULE_AUTO) return fail(SV_ERR_ARG, "unknown fusion rule %d", rule);
    const int cost_prec = precision < 0 ? SV_PREC_FP32 : precision;
    if (max_k == -1 || rule == SV_RULE_AUTO) {
        if (max_k != -1 && (max_k < 1 || max_k > SV_MAX_K)) return fail(SV_ERR_ARG, "max_k %d", max_k);
        if (int rc = choose_plan(g, G, n, SV_C64, cost_prec, rule, max_k, &rule, &max_k)) return rc;
    }
    auto *p = new sv_plan;
    p->n = n;
    p->max_k = max_k;
    p->rule = rule;
    int rc = fuse_gates(g, G, n, max_k, rule, lookup_costs(n, cost_prec, nullptr), p->blocks, true, precision);
    if (rc) {
        delete p;
        return rc;
    }
    *out = p;
    return SV_OK;
}

}  // namespace

extern "C" int sv_fuse(const sv_gate *g, int G, int n, int max_k, int rule, sv_plan **out)
{
    clear_error();
    return fuse_plan(g, G, n, max_k, rule, -1, out);
}

extern "C" int sv_fuse_prec(const sv_gate *g, int G, int n, int max_k, int rule, int precision, sv_plan **out)
{
    clear_error();
    if (precision < 0) return fail(SV_ERR_ARG, "precision %d", precision);
    return fuse_plan(g, G, n, max_k, rule, precision, out);
}

extern "C" int sv_plan_free(sv_plan *p)
{
    delete p;
    return SV_OK;
}

extern "C" int sv_plan_num_blocks(const sv_plan *p, int *out)
{
    clear_error();
    if (!p || !out) return fail(SV_ERR_ARG, "NULL argument");
    *out = int(p->blocks.size());
    return SV_OK;
}

extern "C" int sv_plan_max_k(const sv_plan *p, int *out)
{
    clear_error();
    if (!p || !out) return fail(SV_ERR_ARG, "NULL argument");
    *out = p->max_k;
    return SV_OK;
}

extern "C" int sv_plan_rule(const sv_plan *p, int *out)
{
    clear_error();
    if (!p || !out) return fail(SV_ERR_ARG, "NULL argument");
    *out = p->rule;
    return SV_OK;
}

extern "C" int sv_plan_block(const sv_plan *p, int b, int32_t *k, int32_t *q, int32_t *n_members)
{
    clear_error();
    if (!p) return fail(SV_ERR_ARG, "NULL plan");
    if (b < 0 || b >= int(p->blocks.size())) return fail(SV_ERR_ARG, "block %d out of range", b);
    const Block &B = p->blocks[b];
    if (k) *k = B.k;
    if (q)
        for (int j = 0; j < SV_MAX_K; ++j) q[j] = j < B.k ? B.q[j] : -1;
    if (n_members) *n_members = int(B.members.size());
    return SV_OK;
}

extern "C" int sv_plan_block_pass(const sv_plan *p, int b, int32_t *pass)
{
    clear_error();
    if (!p || !pass) return fail(SV_ERR_ARG, "NULL argument");
    if (b < 0 || b >= int(p->blocks.size())) return fail(SV_ERR_ARG, "block %d out of range", b);
    *pass = p->blocks[b].pass;
    return SV_OK;
}

extern "C" int sv_plan_block_members(const sv_plan *p, int b, int32_t *members)
{
    clear_error();
    if (!p || !members) return fail(SV_ERR_ARG, "NULL argument");
    if (b < 0 || b >= int(p->blocks.size())) return fail(SV_ERR_ARG, "block %d out of range", b);
    const Block &B = p->blocks[b];
    std::copy(B.members.begin(), B.members.end(), members);
    return SV_OK;
}

extern "C" int sv_plan_block_matrix(const sv_plan *p, int b, double *m)
{
    clear_error();
    if (!p || !m) return fail(SV_ERR_ARG, "NULL argument");
    if (b < 0 || b >= int(p->blocks.size())) return fail(SV_ERR_ARG, "block %d out of range", b);
    const Block &B = p->blocks[b];
    std::vector<cd> abi;
    reverse_local_bits(B.m, B.k, abi);
    for (size_t i = 0; i < abi.size(); ++i) {
        m[2 * i] = abi[i].real();
        m[2 * i + 1] = abi[i].imag();
    }
    return SV_OK;
}

extern "C" int sv_apply_plan(sv_state *s, const sv_plan *p, int precision, int use_graph)
{
    clear_error();
    if (int rc = check_state(s)) return rc;
    if (!p) return fail(SV_ERR_ARG, "NULL plan");
    if (int rc = check_precision(s, precision)) return rc;
    for (const auto &b : p->blocks)
        for (int j = 0; j < b.k; ++j)
            if (b.q[j] >= s->n) return fail(SV_ERR_QUBIT, "plan position %d outside a %d-qubit state", b.q[j], s->n);
    if (precision == SV_PREC_SPLIT_FP16)
        for (size_t i = 0; i < p->blocks.size(); ++i) {
            std::string what = "plan block " + std::to_string(i);
            if (int rc = check_unitary(p->blocks[i].m, p->blocks[i].k, what.c_str())) return rc;
        }
    std::vector<Launch> L;
    blocks_to_launches(p->blocks, s, precision, p->rule, L);
    if (int rc = select_device(s)) return rc;
    return run_launches(s, L, use_graph != 0);
}

// ============================================================== circuits
namespace {

// Fuse and apply a validated state's circuit (sv_run_circuit, sv_dm_run).
// basis >= 0: the state first becomes |basis> (sv_run_circuit_basis): the
// first launch produces it itself when it is a tile pass, else it is filled.
int run_circuit_impl(sv_state *s, const sv_gate *g, int G, const sv_run_opts *o, int64_t basis = -1)
{
    sv_run_opts d;
    d.max_k = SV_MAX_K;
    d.precision = s->dtype == SV_C64 ? SV_PREC_FP32 : SV_PREC_FP64;
    d.rule = SV_RULE_NONE;
    d.use_graph = 0;
    if (!o) o = &d;
    if (int rc = check_precision(s, o->precision)) return rc;
    if (int rc = validate_gates(g, G, s->n)) return rc;
    if (o->precision == SV_PREC_SPLIT_FP16)
        if (int rc = check_fp16_gates(g, G)) return rc;
    int max_k = o->max_k, rule = o->rule;
    if (rule < SV_RULE_PAPER || rule > SV_RULE_AUTO) return fail(SV_ERR_ARG, "unknown fusion rule %d", rule);
    if (max_k != -1 && (max_k < 1 || max_k > SV_MAX_K))
        return fail(SV_ERR_ARG, "max_k %d outside 1..%d (or -1)", max_k, SV_MAX_K);
    if (max_k == -1 || rule == SV_RULE_AUTO) {
        if (int rc = choose_plan(g, G, s->n, s->dtype, o->precision, rule, max_k, &rule, &max_k)) return rc;
    }
    std::vector<Block> blocks;
    if (int rc = fuse_gates(g, G, s->n, max_k, rule, lookup_costs(s->n, o->precision, nullptr), blocks, true,
                            o->precision))
        return rc;
    std::vector<Launch> L;
    blocks_to_launches(blocks, s, o->precision, rule, L);
    if (int rc = select_device(s)) return rc;
    if (basis >= 0) {
        // FP32 and split-FP16 tile passes start from the basis state
        // themselves; other first launches get it filled in
        if (!L.empty() && (L[0].path == PATH_TILE || L[0].path == PATH_TILE_FP16))
            L[0].basis = basis;
        else
            SV_HIP(dev::launch_fill_basis(s->dtype, s->buf, s->n, uint64_t(basis), s->stream));
    }
    return run_launches(s, L, o->use_graph != 0);
}

}  // namespace

extern "C" int sv_run_circuit(sv_state *s, const sv_gate *g, int G, const sv_run_opts *o)
{
    clear_error();
    if (int rc = check_state(s)) return rc;
    return run_circuit_impl(s, g, G, o);
}

extern "C" int sv_run_circuit_basis(sv_state *s, uint64_t basis, const sv_gate *g, int G, const sv_run_opts *o)
{
    clear_error();
    if (int rc = check_state(s)) return rc;
    if (basis >> s->n) return fail(SV_ERR_ARG, "basis index %llu >= 2^%d", (unsigned long long)basis, s->n);
    return run_circuit_impl(s, g, G, o, int64_t(basis));
}

// The super circuit is rewritten as a regular circuit of 2n positions
// (dm_expand) and run like any other circuit.
extern "C" int sv_dm_run(sv_state *rho, const sv_gate *g, int G, const sv_super_op *ops, int n_ops,
                         const sv_run_opts *o)
{
    clear_error();
    if (int rc = check_state(rho)) return rc;
    if (rho->n % 2) return fail(SV_ERR_ARG, "a density matrix needs an even number of state qubits, got %d", rho->n);
    if (o && o->precision == SV_PREC_SPLIT_FP16)
        return fail(SV_ERR_ARG, "SV_PREC_SPLIT_FP16 is not available for density matrices (super operators may "
                                "raise the 2-norm its tile passes rely on)");
    if (int rc = validate_gates(g, G, rho->n / 2)) return rc;
    std::vector<sv_gate> full;
    std::vector<std::vector<double>> store;
    if (int rc = dm_expand(g, G, rho->n / 2, ops, n_ops, full, store)) return rc;
    return run_circuit_impl(rho, full.data(), int(full.size()), o);
}

// ============================================================== reductions
namespace {

int read_result(sv_state *s, const double *d_src, size_t count, double *out)
{
    SV_HIP(s->red_host.ensure(count * sizeof(double)));
    SV_HIP(hipMemcpyAsync(s->red_host.p, d_src, count * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    SV_HIP(hipStreamSynchronize(s->stream));
    std::memcpy(out, s->red_host.p, count * sizeof(double));
    return SV_OK;
}

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// Group terms by x mask, stage the tables and upload them into the arena.
// The caller synchronised arena_free and records it after its launches.
int pauli_tables(sv_state *s, const sv_pauli_sum *H, dev::PauliDev &P)
{
    const size_t total = pauli_table_bytes(H);
    SV_HIP(s->stage.ensure(total));
    SV_HIP(s->arena.ensure(total));
    pauli_table_fill(H, static_cast<char *>(s->stage.p), static_cast<const char *>(s->arena.p), P);
    SV_HIP(hipMemcpyAsync(s->arena.p, s->stage.p, total, hipMemcpyHostToDevice, s->stream));
    return SV_OK;
}

}  // namespace

namespace sv {

int check_pauli(const sv_pauli_sum *H, int n)
{
    if (!H) return fail(SV_ERR_ARG, "NULL Pauli sum");
    if (H->n_terms < 0 || H->n_terms > SV_MAX_PAULI_TERMS)
        return fail(SV_ERR_ARG, "Pauli sum with %d terms (0..%d)", H->n_terms, SV_MAX_PAULI_TERMS);
    if (H->reserved != 0) return fail(SV_ERR_ARG, "sv_pauli_sum.reserved must be 0");
    if (H->n_terms && (!H->coef || !H->xmask || !H->zmask)) return fail(SV_ERR_ARG, "NULL Pauli arrays");
    const uint64_t bad = n >= 64 ? 0 : ~((uint64_t(1) << n) - 1);
    for (int t = 0; t < H->n_terms; ++t) {
        if ((H->xmask[t] | H->zmask[t]) & bad) return fail(SV_ERR_QUBIT, "Pauli term %d acts beyond qubit %d", t, n - 1);
        if (!std::isfinite(H->coef[t])) return fail(SV_ERR_ARG, "non-finite Pauli coefficient");
    }
    return SV_OK;
}

namespace {

// Byte offsets of the device tables of a Pauli sum with ng x-mask groups and
// nt terms: group masks, group offsets, term z masks, coefficients, i-powers.
struct PauliLayout {
    size_t gx, goff, tz, tc, tp, total;
    PauliLayout(int ng, int nt)
    {
        gx = 0;
        goff = al256(gx + 8 * std::max(ng, 1));
        tz = al256(goff + 4 * (ng + 1));
        tc = al256(tz + 8 * std::max(nt, 1));
        tp = al256(tc + 8 * std::max(nt, 1));
        total = al256(tp + 4 * std::max(nt, 1));
    }
};

int count_x_groups(const sv_pauli_sum *H)
{
    std::vector<uint64_t> x(H->xmask, H->xmask + H->n_terms);
    std::sort(x.begin(), x.end());
    return int(std::unique(x.begin(), x.end()) - x.begin());
}

}  // namespace

size_t pauli_table_bytes(const sv_pauli_sum *H) { return PauliLayout(count_x_groups(H), H->n_terms).total; }

void pauli_table_fill(const sv_pauli_sum *H, char *h, const char *d, dev::PauliDev &P)
{
    const int nt = H->n_terms;
    std::vector<int> order(nt);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return H->xmask[a] < H->xmask[b]; });
    std::vector<uint64_t> gx;
    std::vector<int32_t> goff;
    for (int i = 0; i < nt; ++i) {
        if (i == 0 || H->xmask[order[i]] != H->xmask[order[i - 1]]) {
            gx.push_back(H->xmask[order[i]]);
            goff.push_back(i);
        }
    }
    goff.push_back(nt);
    const int ng = int(gx.size());
    const PauliLayout L(ng, nt);
    std::memcpy(h + L.gx, gx.data(), 8 * ng);
    std::memcpy(h + L.goff, goff.data(), 4 * (ng + 1));
    for (int i = 0; i < nt; ++i) {
        const int t = order[i];
        reinterpret_cast<uint64_t *>(h + L.tz)[i] = H->zmask[t];
        reinterpret_cast<double *>(h + L.tc)[i] = H->coef[t];
        reinterpret_cast<int32_t *>(h + L.tp)[i] = __builtin_popcountll(H->xmask[t] & H->zmask[t]) & 3;
    }
    P.n_groups = ng;
    P.gx = reinterpret_cast<const uint64_t *>(d + L.gx);
    P.goff = reinterpret_cast<const int32_t *>(d + L.goff);
    P.tz = reinterpret_cast<const uint64_t *>(d + L.tz);
    P.tc = reinterpret_cast<const double *>(d + L.tc);
    P.tpow = reinterpret_cast<const int32_t *>(d + L.tp);
}

}  // namespace sv

extern "C" int sv_norm(sv_state *s, double *out)
{
    clear_error();
    if (int rc = check_state(s)) return rc;
    if (!out) return fail(SV_ERR_ARG, "NULL out");
    if (int rc = select_device(s)) return rc;
    double *part = static_cast<double *>(s->red.p);
    double *res = part + 2 * dev::kRedBlocks;
    {
        LaunchTimer t(stat_class(FAM_REDUCE, 1), s->stream);
        SV_HIP(dev::launch_norm(s->dtype, s->buf, s->n, part, res, s->stream));
    }
    return read_result(s, res, 1, out);
}

extern "C" int sv_inner(sv_state *a, sv_state *b, double *re, double *im)
{
    clear_error();
    if (!a || !b || !re || !im) return fail(SV_ERR_ARG, "NULL argument");
    if (a->n != b->n) return fail(SV_ERR_ARG, "qubit counts differ (%d vs %d)", a->n, b->n);
    if (int rc = select_device(b)) return rc;
    if (int rc = stream_after(b->stream, a->stream)) return rc;
    double *part = static_cast<double *>(b->red.p);
    double *res = part + 2 * dev::kRedBlocks;
    {
        LaunchTimer t(stat_class(FAM_REDUCE, 2), b->stream);
        SV_HIP(dev::launch_inner(a->dtype, a->buf, b->dtype, b->buf, b->n, part, res, b->stream));
    }
    double v[2];
    if (int rc = read_result(b, res, 2, v)) return rc;
    *re = v[0];
    *im = v[1];
    return SV_OK;
}

extern "C" int sv_expectation(sv_state *s, const sv_pauli_sum *H, double *out)
{
    clear_error();
    if (int rc = check_state(s)) return rc;
    if (!out) return fail(SV_ERR_ARG, "NULL out");
    if (int rc = check_pauli(H, s->n)) return rc;
    if (H->n_terms == 0) {
        *out = 0.0;
        return SV_OK;
    }
    if (int rc = select_device(s)) return rc;
    SV_HIP(hipEventSynchronize(s->arena_free));
    dev::PauliDev P;
    if (int rc = pauli_tables(s, H, P)) return rc;
    double *part = static_cast<double *>(s->red.p);
    double *res = part + 2 * dev::kRedBlocks;
    {
        LaunchTimer t(stat_class(FAM_REDUCE, 3), s->stream);
        SV_HIP(dev::launch_pauli_expect(s->dtype, s->buf, s->n, P, part, res, s->stream));
    }
    SV_HIP(hipEventRecord(s->arena_free, s->stream));
    return read_result(s, res, 1, out);
}

extern "C" int sv_dm_expectation(sv_state *rho, const sv_pauli_sum *H, double *out)
{
    clear_error();
    if (int rc = check_state(rho)) return rc;
    if (!out) return fail(SV_ERR_ARG, "NULL out");
    if (rho->n % 2) return fail(SV_ERR_ARG, "a density matrix needs an even number of state qubits, got %d", rho->n);
    const int n = rho->n / 2;
    if (int rc = check_pauli(H, n)) return rc;
    if (H->n_terms == 0) {
        *out = 0.0;
        return SV_OK;
    }
    if (int rc = select_device(rho)) return rc;
    SV_HIP(hipEventSynchronize(rho->arena_free));
    dev::PauliDev P;
    if (int rc = pauli_tables(rho, H, P)) return rc;
    double *part = static_cast<double *>(rho->red.p);
    double *res = part + 2 * dev::kRedBlocks;
    {
        LaunchTimer t(stat_class(FAM_REDUCE, 5), rho->stream);
        SV_HIP(dev::launch_dm_expect(rho->dtype, rho->buf, n, P, part, res, rho->stream));
    }
    SV_HIP(hipEventRecord(rho->arena_free, rho->stream));
    return read_result(rho, res, 1, out);
}

namespace {

// p[i] = ||K_i psi||^2 (FP64; one pass over the state per kMaxKraus
// operators).  Synchronises.
int kraus_weights(sv_state *s, const KrausSet &ks, double *p)
{
    if (int rc = select_device(s)) return rc;
    constexpr int kChunks = (kMaxKrausOps + dev::kMaxKraus - 1) / dev::kMaxKraus;
    SV_HIP(s->red.ensure(sizeof(double) * (size_t(dev::kMaxKraus) * dev::kRedBlocks + dev::kMaxKraus * kChunks)));
    SV_HIP(hipEventSynchronize(s->arena_free));
    const size_t bytes = sizeof(cd) * ks.canon.size();
    SV_HIP(s->stage.ensure(bytes));
    SV_HIP(s->arena.ensure(bytes));
    std::memcpy(s->stage.p, ks.canon.data(), bytes);
    SV_HIP(hipMemcpyAsync(s->arena.p, s->stage.p, bytes, hipMemcpyHostToDevice, s->stream));
    double *part = static_cast<double *>(s->red.p);
    double *res = part + size_t(dev::kMaxKraus) * dev::kRedBlocks;
    const size_t D2 = size_t(1) << (2 * ks.k);
    for (int c0 = 0; c0 < ks.n_ops; c0 += dev::kMaxKraus) {
        dev::KrausDev K;
        K.n_ops = std::min(dev::kMaxKraus, ks.n_ops - c0);
        K.k = ks.k;
        for (int j = 0; j < 3; ++j) K.pos[j] = j < ks.k ? ks.sorted_q[j] : 0;
        K.m = static_cast<const double *>(s->arena.p) + 2 * D2 * c0;
        LaunchTimer t(stat_class(FAM_REDUCE, 6), s->stream);
        SV_HIP(dev::launch_kraus_probs(s->dtype, s->buf, s->n, K, part, res + c0, s->stream));
    }
    SV_HIP(hipEventRecord(s->arena_free, s->stream));
    return read_result(s, res, size_t(ks.n_ops), p);
}

// Draw one Kraus operator with probability p_i / sum p by the uniform u and
// apply K_i / sqrt(p_i).  The first i whose running sum exceeds u * sum p is
// taken (zero-weight operators are never taken).
int sample_kraus(sv_state *s, const sv_super_op &op, double u, int32_t *chosen, double *p_chosen)
{
    KrausSet ks;
    if (int rc = kraus_canonical(op, s->n, ks)) return rc;
    double p[kMaxKrausOps];
    if (int rc = kraus_weights(s, ks, p)) return rc;
    double total = 0.0;
    for (int i = 0; i < ks.n_ops; ++i) total += p[i];
    if (!(total > 0.0) || !std::isfinite(total)) return fail(SV_ERR_ARG, "Kraus outcome weights sum to %g", total);
    int pick = -1;
    double run = 0.0;
    for (int i = 0; i < ks.n_ops; ++i) {
        run += p[i];
        if (p[i] > 0.0) pick = i;  // the last nonzero one, should rounding leave u * total above every sum
        if (p[i] > 0.0 && u * total < run) break;
    }
    const size_t D = size_t(1) << ks.k;
    const double scale = 1.0 / std::sqrt(p[pick]);
    std::vector<double> m(2 * D * D);
    for (size_t e = 0; e < 2 * D * D; ++e) m[e] = ks.abi[2 * D * D * pick + e] * scale;
    sv_gate h{};
    h.kind = SV_G_MATRIX;
    h.k = ks.k;
    h.param = -1;
    for (int a = 0; a < ks.k; ++a) h.q[a] = ks.q[a];
    h.m = m.data();
    if (int rc = apply_gate_impl(s, &h)) return rc;
    if (chosen) *chosen = pick;
    if (p_chosen) *p_chosen = p[pick] / total;
    return SV_OK;
}

}  // namespace

extern "C" int sv_kraus_probabilities(sv_state *s, const sv_super_op *op, double *p_out)
{
    clear_error();
    if (int rc = check_state(s)) return rc;
    if (!op || !p_out) return fail(SV_ERR_ARG, "NULL argument");
    KrausSet ks;
    if (int rc = kraus_canonical(*op, s->n, ks)) return rc;
    if (int rc = kraus_weights(s, ks, p_out)) return rc;
    for (int i = ks.n_ops; i < op->n_left; ++i) p_out[i] = 0.0;
    return SV_OK;
}

extern "C" int sv_apply_kraus_sampled(sv_state *s, const sv_super_op *op, double u, int32_t *chosen,
                                      double *p_chosen)
{
    clear_error();
    if (int rc = check_state(s)) return rc;
    if (!op) return fail(SV_ERR_ARG, "NULL operator");
    if (!(u >= 0.0 && u < 1.0)) return fail(SV_ERR_ARG, "uniform %g outside [0, 1)", u);
    return sample_kraus(s, *op, u, chosen, p_chosen);
}

extern "C" int sv_run_trajectory(sv_state *s, const sv_gate *g, int G, const sv_super_op *ops, int n_ops,
                                 const double *uniforms, const sv_run_opts *o, int32_t *outcomes)
{
    clear_error();
    if (int rc = check_state(s)) return rc;
    if (int rc = validate_gates(g, G, s->n)) return rc;
    if (n_ops < 0 || (n_ops && (!ops || !uniforms))) return fail(SV_ERR_ARG, "NULL operator or uniform array");
    for (int j = 0; j < n_ops; ++j) {
        KrausSet ks;
        if (int rc = kraus_canonical(ops[j], s->n, ks)) return rc;
        if (ops[j].after < 0 || ops[j].after > G || (j && ops[j].after < ops[j - 1].after))
            return fail(SV_ERR_ARG, "operator %d: after = %d out of order (0..%d, nondecreasing)", j, ops[j].after, G);
        if (!(uniforms[j] >= 0.0 && uniforms[j] < 1.0))
            return fail(SV_ERR_ARG, "uniform %d = %g outside [0, 1)", j, uniforms[j]);
    }
    int done = 0;
    for (int j = 0; j <= n_ops; ++j) {
        const int upto = j < n_ops ? ops[j].after : G;
        if (upto > done) {
            if (int rc = run_circuit_impl(s, g + done, upto - done, o)) return rc;
            done = upto;
        }
        if (j < n_ops) {
            int32_t pick = -1;
            if (int rc = sample_kraus(s, ops[j], uniforms[j], &pick, nullptr)) return rc;
            if (outcomes) outcomes[j] = pick;
        }
    }
    return SV_OK;
}

// ============================================================== projections, measurement, control
extern "C" int sv_project(sv_state *s, int k, const int32_t *q, uint64_t bits, int renormalize, double *prob)
{
    clear_error();
    if (int rc = check_state(s)) return rc;
    if (k < 1 || k > SV_MAX_K || !q) return fail(SV_ERR_ARG, "projection on %d qubits (1..%d)", k, SV_MAX_K);
    if (bits >> k) return fail(SV_ERR_ARG, "bits 0x%llx exceed %d qubits", (unsigned long long)bits, k);
    sv_gate h{};
    h.kind = SV_G_MATRIX;
    h.k = k;
    h.param = -1;
    for (int j = 0; j < k; ++j) h.q[j] = q[j];
    if (int rc = check_gate_qubits(h, s->n)) return rc;
    // |bits><bits| on q (q[0] the most significant bit of bits)
    const size_t D = size_t(1) << k;
    std::vector<double> m(2 * D * D, 0.0);
    m[2 * (bits * D + bits)] = 1.0;
    h.m = m.data();
    if (int rc = select_device(s)) return rc;
    if (int rc = apply_gate_impl(s, &h)) return rc;
    double p = 0.0;
    if (int rc = sv_norm(s, &p)) return rc;
    if (renormalize) {
        if (!(p > 0.0)) return fail(SV_ERR_ARG, "the projection has probability 0; cannot renormalise");
        const double c = 1.0 / std::sqrt(p);
        const double sc[8] = {c, 0, 0, 0, 0, 0, c, 0};  // c I on q[0]
        sv_gate t{};
        t.kind = SV_G_MATRIX;
        t.k = 1;
        t.q[0] = q[0];
        t.param = -1;
        t.m = sc;
        if (int rc = apply_gate_impl(s, &t)) return rc;
    }
    if (prob) *prob = p;
    return SV_OK;
}

extern "C" int sv_measure(sv_state *s, int k, const int32_t *q, const double *uniforms, uint64_t *bits,
                          double *prob)
{
    clear_error();
    if (int rc = check_state(s)) return rc;
    if (k < 1 || k > s->n || !q || !uniforms) return fail(SV_ERR_ARG, "measurement of %d qubits", k);
    for (int j = 0; j < k; ++j) {
        if (q[j] < 0 || q[j] >= s->n) return fail(SV_ERR_QUBIT, "qubit %d outside 0..%d", q[j], s->n - 1);
        for (int i = 0; i < j; ++i)
            if (q[i] == q[j]) return fail(SV_ERR_QUBIT, "qubit %d repeated", q[j]);
        if (!(uniforms[j] >= 0.0 && uniforms[j] < 1.0))
            return fail(SV_ERR_ARG, "uniform %d = %g outside [0, 1)", j, uniforms[j]);
    }
    // qubit by qubit: the Kraus set {|0><0|, |1><1|} sampled with uniforms[j]
    static const double proj[16] = {1, 0, 0, 0, 0, 0, 0, 0,   // |0><0|
                                    0, 0, 0, 0, 0, 0, 1, 0};  // |1><1|
    uint64_t out = 0;
    double ptot = 1.0;
    for (int j = 0; j < k; ++j) {
        sv_super_op op{};
        op.after = 0;
        op.k = 1;
        op.q[0] = q[j];
        op.n_left = op.n_right = 2;
        op.left = op.right = proj;
        int32_t b = 0;
        double pb = 0.0;
        if (int rc = sample_kraus(s, op, uniforms[j], &b, &pb)) return rc;
        out = (out << 1) | uint64_t(b);
        ptot *= pb;
    }
    if (bits) *bits = out;
    if (prob) *prob = ptot;
    return SV_OK;
}

extern "C" int sv_controlled_gate(const sv_gate *g, int n_c, const int32_t *controls, sv_gate *out, double *m_out)
{
    clear_error();
    if (!g || !out || !m_out || (n_c > 0 && !controls)) return fail(SV_ERR_ARG, "NULL argument");
    if (int rc = check_gate_shape(*g)) return rc;
    if (n_c < 1 || n_c + g->k > SV_MAX_K)
        return fail(SV_ERR_ARG, "%d controls on a %d-qubit gate (at most %d qubits in all)", n_c, g->k, SV_MAX_K);
    sv_gate h{};
    h.kind = SV_G_MATRIX;
    h.k = n_c + g->k;
    h.param = -1;
    for (int j = 0; j < n_c; ++j) h.q[j] = controls[j];
    for (int j = 0; j < g->k; ++j) h.q[n_c + j] = g->q[j];
    if (int rc = check_gate_qubits(h, 64)) return rc;
    std::vector<cd> U;
    if (int rc = gate_matrix_abi(*g, U)) return rc;
    // identity, except the block where every control (the most significant
    // local bits) is 1, which holds U
    const size_t D = size_t(1) << h.k, d = size_t(1) << g->k, off = D - d;
    std::fill(m_out, m_out + 2 * D * D, 0.0);
    for (size_t i = 0; i < off; ++i) m_out[2 * (i * D + i)] = 1.0;
    for (size_t r = 0; r < d; ++r)
        for (size_t c = 0; c < d; ++c) {
            m_out[2 * ((off + r) * D + off + c)] = U[r * d + c].real();
            m_out[2 * ((off + r) * D + off + c) + 1] = U[r * d + c].imag();
        }
    h.m = m_out;
    *out = h;
    return SV_OK;
}

extern "C" int sv_apply_pauli_sum(sv_state *psi, const sv_pauli_sum *H, sv_state *out)
{
    clear_error();
    if (!psi || !out) return fail(SV_ERR_ARG, "NULL state handle");
    if (psi == out) return fail(SV_ERR_ARG, "output must be a different state");
    if (psi->n != out->n || psi->dtype != out->dtype) return fail(SV_ERR_ARG, "states differ in n or type");
    if (int rc = check_pauli(H, psi->n)) return rc;
    if (int rc = select_device(psi)) return rc;
    if (int rc = stream_after(psi->stream, out->stream)) return rc;
    SV_HIP(hipEventSynchronize(psi->arena_free));
    dev::PauliDev P;
    if (H->n_terms == 0) {
        SV_HIP(dev::launch_fill_basis(out->dtype, out->buf, out->n, ~uint64_t(0), psi->stream));
    } else {
        if (int rc = pauli_tables(psi, H, P)) return rc;
        LaunchTimer t(stat_class(FAM_REDUCE, 4), psi->stream);
        SV_HIP(dev::launch_pauli_apply(psi->dtype, psi->buf, out->buf, psi->n, P, psi->stream));
    }
    SV_HIP(hipEventRecord(psi->arena_free, psi->stream));
    if (int rc = stream_after(out->stream, psi->stream)) return rc;
    return SV_OK;
}

// ============================================================== adjoint
namespace {

// One step of the backward sweep (gates are visited from last to first).
struct BwdStep {
    enum Kind { SINGLE, RUN, UNDO } kind;
    int gate = -1;        // SINGLE: the gate
    int slot = -1;        // SINGLE: gradient slot or -1; RUN: first slot
    int n_terms = 0;      // RUN: rotations in the run
    uint64_t x[dev::kMaxGradTerms] = {}, z[dev::kMaxGradTerms] = {};
    int pw[dev::kMaxGradTerms] = {};
    size_t l0 = 0, l1 = 0;  // RUN / UNDO: launches [l0, l1) that undo the gates
};

// Fuse the daggers of gates hi, hi-1, .., lo (in that order) into blocks and
// append their launches.
int dagger_launches(const sv_gate *g, int hi, int lo, const sv_state *s, int prec, std::vector<Launch> &out)
{
    const int cnt = hi - lo + 1;
    std::vector<sv_gate> dg(cnt);
    std::vector<std::vector<double>> store(cnt);
    int kmax = 1;
    for (int t = 0; t < cnt; ++t) {
        const sv_gate &src = g[hi - t];
        std::vector<cd> m;
        if (int rc = gate_matrix_abi(src, m)) return rc;
        const int D = 1 << src.k;
        store[t].resize(2 * size_t(D) * D);
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) {
                const cd v = std::conj(m[size_t(c) * D + r]);
                store[t][2 * (size_t(r) * D + c)] = v.real();
                store[t][2 * (size_t(r) * D + c) + 1] = v.imag();
            }
        sv_gate d = src;
        d.kind = SV_G_MATRIX;
        d.param = -1;
        d.m = store[t].data();
        dg[t] = d;
        kmax = std::max(kmax, src.k);
    }
    std::vector<Block> blocks;
    const CostTable cost = lookup_costs(s->n, prec, nullptr);
    // The plan of a run (dense blocks of the cheapest k, or tile passes)
    // depends on its gates' positions and the cost table only; it is
    // remembered per run structure, so a sweep with new angles only forms
    // the block matrices.  A colliding entry can only name another valid plan.
    uint64_t key = 1469598103934665603ull;
    auto mix = [&key](uint64_t v) { key = (key ^ v) * 1099511628211ull; };
    mix(uint64_t(s->n));
    mix(uint64_t(s->dtype));
    mix(uint64_t(prec));
    mix(cost_version());
    mix(uint64_t(tile_union_limit()));
    mix(uint64_t(tile_pass_bits()) | uint64_t(tile_pass_capacity(prec)) << 8);
    mix(uint64_t(cnt));
    for (int t = 0; t < cnt; ++t) {
        mix(uint64_t(dg[t].k));
        for (int j = 0; j < dg[t].k; ++j) mix(uint64_t(dg[t].q[j]));
    }
    static std::mutex memo_mu;
    static std::unordered_map<uint64_t, int> memo;  // k of the dense plan, or 0 for tile passes
    int choice = -1;
    {
        std::lock_guard<std::mutex> lk(memo_mu);
        auto it = memo.find(key);
        if (it != memo.end() && (it->second == 0 ? kmax <= 4 : it->second >= kmax)) choice = it->second;
    }
    if (choice < 0) {
        // block size: the cheapest plan under the cost table (complex64
        // blocks of 4..6 qubits run on MFMA; complex128 stays at 4), or
        // tile passes of <= 4-qubit blocks (one launch for both states per
        // pass) where the cost table prices them lower
        int kbest = std::max(kmax, 4);
        double best = 1e300;
        if (s->dtype == SV_C64 && s->n >= 11) {
            for (int k = std::max(kmax, 4); k <= SV_MAX_K; ++k) {
                if (int rc = fuse_gates(dg.data(), cnt, s->n, k, SV_RULE_ENHANCED, cost, blocks, false)) return rc;
                const double c = plan_cost(blocks, cost);
                if (c < best - 1e-12) {
                    best = c;
                    kbest = k;
                }
            }
        }
        choice = kbest;
        if (s->dtype == SV_C64 && kmax <= 4 && dev::tile_supported(s->n, 4)) {
            if (best > 1e299) {
                if (int rc = fuse_gates(dg.data(), cnt, s->n, kbest, SV_RULE_ENHANCED, cost, blocks, false)) return rc;
                best = plan_cost(blocks, cost);
            }
            if (int rc = fuse_gates(dg.data(), cnt, s->n, 4, SV_RULE_TILED, cost, blocks, false, prec)) return rc;
            if (tiled_plan_cost(blocks, s->n, cost) < best - 1e-12) choice = 0;
        }
        std::lock_guard<std::mutex> lk(memo_mu);
        if (memo.size() > 65536) memo.clear();
        memo[key] = choice;
    }
    if (choice == 0) {
        if (int rc = fuse_gates(dg.data(), cnt, s->n, 4, SV_RULE_TILED, cost, blocks, true, prec)) return rc;
        std::vector<Launch> tl;
        group_tile_passes(blocks, s->n, prec, tl);
        for (auto &L : tl) out.push_back(std::move(L));
        return SV_OK;
    }
    const int kbest = choice;
    if (int rc = fuse_gates(dg.data(), cnt, s->n, kbest, SV_RULE_ENHANCED, cost, blocks)) return rc;
    for (const auto &b : blocks) {
        Launch L;
        L.k = b.k;
        std::copy(b.q, b.q + SV_MAX_K, L.q);
        L.path = choose_path(s->dtype, prec, b.k, b.q, s->n);
        L.m = b.m;
        out.push_back(std::move(L));
    }
    return SV_OK;
}

}  // namespace

namespace {

int backward_impl(sv_state *psi, sv_state *scratch, const sv_gate *g, int G, const sv_pauli_sum *H, double *grad,
                  int n_params, int prec);

}  // namespace

extern "C" int sv_backward(sv_state *psi, sv_state *scratch, const sv_gate *g, int G, const sv_pauli_sum *H,
                           double *grad, int n_params)
{
    clear_error();
    if (!psi) return fail(SV_ERR_ARG, "NULL state handle");
    return backward_impl(psi, scratch, g, G, H, grad, n_params, psi->dtype == SV_C64 ? SV_PREC_FP32 : SV_PREC_FP64);
}

extern "C" int sv_backward_prec(sv_state *psi, sv_state *scratch, const sv_gate *g, int G, const sv_pauli_sum *H,
                                double *grad, int n_params, int precision)
{
    clear_error();
    if (!psi) return fail(SV_ERR_ARG, "NULL state handle");
    if (int rc = check_precision(psi, precision)) return rc;
    return backward_impl(psi, scratch, g, G, H, grad, n_params, precision);
}

namespace {

int backward_impl(sv_state *psi, sv_state *scratch, const sv_gate *g, int G, const sv_pauli_sum *H, double *grad,
                  int n_params, int prec)
{
    if (!psi || !scratch) return fail(SV_ERR_ARG, "NULL state handle");
    if (psi == scratch) return fail(SV_ERR_ARG, "scratch must be a different state");
    if (psi->n != scratch->n || psi->dtype != scratch->dtype) return fail(SV_ERR_ARG, "states differ in n or type");
    if (n_params < 0 || (n_params > 0 && !grad)) return fail(SV_ERR_ARG, "bad gradient buffer");
    if (int rc = validate_gates(g, G, psi->n)) return rc;
    if (prec == SV_PREC_SPLIT_FP16)
        if (int rc = check_fp16_gates(g, G)) return rc;
    if (int rc = check_pauli(H, psi->n)) return rc;
    for (int i = 0; i < G; ++i)
        if (g[i].param >= n_params) return fail(SV_ERR_ARG, "gate %d: param %d >= n_params %d", i, g[i].param, n_params);

    // plan the sweep: runs of rotations on distinct qubits share one gradient
    // pass (they commute, so each sees the same phi and lam); runs of
    // non-parameterised gates are undone as fused dagger blocks
    std::vector<BwdStep> steps;
    std::vector<Launch> launches;
    std::vector<int> slot_param;
    struct RunJob {
        int hi, lo;
        size_t step;
    };
    std::vector<RunJob> jobs;  // dagger runs: gates hi..lo, undone at steps[step]
    int i = G - 1;
    while (i >= 0) {
        if (g[i].param >= 0) {
            uint64_t used = 0;
            int j = i;
            while (j >= 0 && g[j].param >= 0 && g[j].k == 1 && !((used >> g[j].q[0]) & 1) &&
                   i - j < dev::kMaxGradTerms) {
                used |= uint64_t(1) << g[j].q[0];
                --j;
            }
            if (i - j >= 2) {
                BwdStep st;
                st.kind = BwdStep::RUN;
                st.slot = int(slot_param.size());
                for (int t = i; t > j; --t) {
                    const uint64_t b = uint64_t(1) << g[t].q[0];
                    const int e = st.n_terms++;
                    st.x[e] = g[t].kind == SV_G_RZ ? 0 : b;
                    st.z[e] = g[t].kind == SV_G_RX ? 0 : b;
                    st.pw[e] = g[t].kind == SV_G_RY ? 1 : 0;
                    slot_param.push_back(g[t].param);
                }
                jobs.push_back({i, j + 1, steps.size()});
                steps.push_back(st);
                i = j;
                continue;
            }
            BwdStep st;
            st.kind = BwdStep::SINGLE;
            st.gate = i;
            st.slot = int(slot_param.size());
            slot_param.push_back(g[i].param);
            steps.push_back(st);
            --i;
            continue;
        }
        int j = i;
        while (j >= 0 && g[j].param < 0) --j;
        if (i - j == 1 && g[i].k <= 2) {
            BwdStep st;
            st.kind = BwdStep::SINGLE;
            st.gate = i;
            steps.push_back(st);
            --i;
            continue;
        }
        BwdStep st;
        st.kind = BwdStep::UNDO;
        jobs.push_back({i, j + 1, steps.size()});
        steps.push_back(st);
        i = j;
    }
    // the dagger blocks of the runs are independent host work: spread over
    // threads, then appended in sweep order
    {
        std::vector<std::vector<Launch>> outs(jobs.size());
        std::vector<int> rcs(jobs.size(), SV_OK);
        std::vector<std::string> msgs(jobs.size());
        std::atomic<size_t> next(0);
        auto worker = [&]() {
            for (size_t t; (t = next.fetch_add(1)) < jobs.size();) {
                rcs[t] = dagger_launches(g, jobs[t].hi, jobs[t].lo, psi, prec, outs[t]);
                if (rcs[t]) msgs[t] = last_error_cstr();
            }
        };
        const unsigned hw = std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
        const unsigned nt = jobs.size() >= 16 ? std::min<unsigned>(hw, unsigned(jobs.size() / 4)) : 1u;
        std::vector<std::thread> pool;
        for (unsigned t = 1; t < nt; ++t) pool.emplace_back(worker);
        worker();
        for (auto &th : pool) th.join();
        for (size_t t = 0; t < jobs.size(); ++t) {
            if (rcs[t]) return fail(rcs[t], "%s", msgs[t].c_str());
            BwdStep &st = steps[jobs[t].step];
            st.l0 = launches.size();
            for (auto &L : outs[t]) launches.push_back(std::move(L));
            st.l1 = launches.size();
        }
    }
    const int slots = int(slot_param.size());

    if (int rc = select_device(psi)) return rc;
    // lam <- H psi on psi's stream
    if (int rc = sv_apply_pauli_sum(psi, H, scratch)) return rc;
    SV_HIP(hipEventSynchronize(psi->arena_free));
    const size_t bytes = pack_operands(launches, psi->dtype, psi->stage);
    if (bytes == size_t(-1)) return fail(SV_ERR_HIP, "pinned staging allocation failed");
    if (bytes) {
        SV_HIP(psi->arena.ensure(bytes));
        SV_HIP(hipMemcpyAsync(psi->arena.p, psi->stage.p, bytes, hipMemcpyHostToDevice, psi->stream));
    }
    const size_t part_doubles = size_t(std::max(slots, 1)) * dev::kRedBlocks * 2;
    SV_HIP(psi->grad.ensure((part_doubles + 2 * size_t(std::max(slots, 1))) * sizeof(double)));
    double *part = static_cast<double *>(psi->grad.p);
    double *sums = part + part_doubles;
    for (const BwdStep &st : steps) {
        if (st.kind == BwdStep::SINGLE) {
            const sv_gate &gg = g[st.gate];
            std::vector<cd> m, mdag;
            int sq[SV_MAX_K];
            if (int rc = gate_matrix_canonical(gg, m, sq)) return rc;
            const int D = 1 << gg.k;
            mdag.resize(m.size());
            for (int r = 0; r < D; ++r)
                for (int c = 0; c < D; ++c) mdag[size_t(r) * D + c] = std::conj(m[size_t(c) * D + r]);
            const int pauli = st.slot < 0 ? 0 : gg.kind == SV_G_RX ? 1 : gg.kind == SV_G_RY ? 2 : 3;
            LaunchTimer t(stat_class(FAM_ADJOINT, gg.k), psi->stream);
            SV_HIP(dev::launch_backward_step(psi->dtype, gg.k, sq, mdag.data(), pauli, psi->buf, scratch->buf, psi->n,
                                             part, st.slot, psi->stream));
            continue;
        }
        if (st.kind == BwdStep::RUN) {
            LaunchTimer t(stat_class(FAM_ADJOINT, 3), psi->stream);
            SV_HIP(dev::launch_grad_terms(psi->dtype, st.n_terms, st.x, st.z, st.pw, psi->buf, scratch->buf, psi->n,
                                          part, st.slot, psi->stream));
        }
        const Launch *sub = launches.data() + st.l0;
        const size_t cnt = st.l1 - st.l0;
        if (int rc = enqueue(sub, cnt, psi->dtype, psi->buf, psi->n, psi->arena.p, psi->stream, scratch->buf)) return rc;
    }
    SV_HIP(hipEventRecord(psi->arena_free, psi->stream));
    if (slots) {
        SV_HIP(dev::launch_sum_partials(part, slots, sums, psi->stream));
        std::vector<double> h(2 * size_t(slots));
        if (int rc = read_result(psi, sums, h.size(), h.data())) return rc;
        for (int sl = 0; sl < slots; ++sl) grad[slot_param[sl]] += h[2 * sl + 1];  // Im <lam|P|phi>
    } else {
        SV_HIP(hipStreamSynchronize(psi->stream));
    }
    if (int rc = stream_after(scratch->stream, psi->stream)) return rc;
    return SV_OK;
}

}  // namespace

// ============================================================== stats
extern "C" int sv_stats_enable(int on)
{
    clear_error();
    return stats_enable(on);
}
extern "C" int sv_stats_reset(void)
{
    clear_error();
    return stats_reset();
}
extern "C" int sv_stats_query(int cls, int64_t *launches, double *total_ms)
{
    clear_error();
    if (!launches || !total_ms) return fail(SV_ERR_ARG, "NULL argument");
    return stats_query(cls, launches, total_ms);
}

extern "C" int sv_graph_stats(const sv_state *s, int64_t *runs, int64_t *reused)
{
    clear_error();
    if (int rc = check_state(s)) return rc;
    if (runs) *runs = s->graph_launches;
    if (reused) *reused = s->graph_updates;
    return SV_OK;
}
