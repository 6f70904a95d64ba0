// Batched noisy trajectories of uneven qubit counts.
//
// The paper's Simulations with noise section evolves pure states with noise
// channels sampled into the circuit ("sampling of the Kraus operators") to
// reach larger systems than density matrices allow.  Here every trajectory
// is an independent circuit (its noise draws already materialised as Pauli
// gates) run from |0..0>, and <Z_0> is reported per trajectory.
//
// Schedule (built once at creation, replayable as one hipGraph):
//   * SMALL trajectories (n <= 13, state <= 64 KiB) run entirely in LDS: one
//     persistent workgroup takes trajectories in turn, applies every fused
//     block of it in LDS, reduces <Z_0> in FP64 and writes the final state
//     out once.  No HBM traffic per gate.
//   * LARGE trajectories (n >= 14) are planned with the tiled rule (passes of
//     several <= 4-qubit blocks, one read and one write of the state each,
//     FP32 or split BF16 / FP16 products by the batch's precision)
//     and advance in lock step: launch s runs pass s of every large
//     trajectory that has one, as tile ranges of a shared grid (one tile
//     kernel, per-pass layouts and operands read from device tables).  <Z_0>
//     is then reduced in fixed-size chunks and summed per trajectory in a
//     fixed order (FP64).
//   * the small-trajectory kernel and the large-trajectory chain are
//     independent and are captured on two forked streams, so they overlap.
// The fusion limit is chosen per batch: with max_k = -1 the batch is timed
// with k = 2, 3 and 4 at creation and the fastest schedule is kept.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>

#include "runtime.h"

using namespace sv;

namespace {

constexpr int kSmallMaxN = 13;
constexpr int kThreads = 256;
constexpr int kZ0ChunkBits = 16;  // amplitudes per <Z_0> partial sum (2^16)

struct BBlock {
    uint64_t state_off;  // complex elements from the start of the batch buffer
    int32_t n;
    int32_t k;
    int32_t q[SV_MAX_K];  // ascending
    int32_t mat_off;      // float2 index into the matrix pool (canonical order)
    int32_t lm;           // which of positions 0, 1 are targets (bit mask)
    int32_t kh;           // number of targets at positions >= 2
    int32_t hp[4];        // those positions, ascending
};

struct BSmall {
    uint64_t state_off;
    int32_t n;
    int32_t first_block;
    int32_t n_blocks;
    int32_t out;
};

struct BLarge {
    uint64_t state_off;
    int32_t n;
    int32_t out;
    int32_t zfirst;  // first <Z_0> chunk of the trajectory
    int32_t zcount;  // its number of chunks
};

struct BZUnit {
    uint64_t off;    // complex elements from the start of the batch buffer (even)
    uint32_t count;
    uint32_t pad;
};

__device__ __forceinline__ uint64_t ins0b(uint64_t x, int p)
{
    return ((x >> p) << (p + 1)) | (x & ((uint64_t(1) << p) - 1));
}

// Apply one k-qubit block to group g of a state (generic gather / scatter).
template <int K>
__device__ __forceinline__ void apply_group(float2 *__restrict__ st, const BBlock &b, const float2 *__restrict__ m,
                                            uint64_t g)
{
    constexpr int D = 1 << K;
    uint64_t base = g;
#pragma unroll
    for (int j = 0; j < K; ++j) base = ins0b(base, b.q[j]);
    float vr[D], vi[D];
#pragma unroll
    for (int mm = 0; mm < D; ++mm) {
        uint64_t o = base;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if ((mm >> j) & 1) o += uint64_t(1) << b.q[j];
        const float2 v = st[o];
        vr[mm] = v.x;
        vi[mm] = v.y;
    }
#pragma unroll
    for (int mm = 0; mm < D; ++mm) {
        float sr = 0.f, si = 0.f;
#pragma unroll
        for (int mp = 0; mp < D; ++mp) {
            const float2 a = m[mm * D + mp];
            sr = fmaf(a.x, vr[mp], sr);
            sr = fmaf(-a.y, vi[mp], sr);
            si = fmaf(a.x, vi[mp], si);
            si = fmaf(a.y, vr[mp], si);
        }
        uint64_t o = base;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if ((mm >> j) & 1) o += uint64_t(1) << b.q[j];
        st[o] = make_float2(sr, si);
    }
}

__device__ __forceinline__ void apply_group_k(float2 *st, const BBlock &b, const float2 *m, uint64_t g)
{
    switch (b.k) {
    case 1: apply_group<1>(st, b, m, g); break;
    case 2: apply_group<2>(st, b, m, g); break;
    case 3: apply_group<3>(st, b, m, g); break;
    case 4: apply_group<4>(st, b, m, g); break;
    case 5: apply_group<5>(st, b, m, g); break;
    default: apply_group<6>(st, b, m, g); break;
    }
}

__device__ double block_sum(double v)
{
    __shared__ double sh[kThreads];
    const int t = threadIdx.x;
    __syncthreads();
    sh[t] = v;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// One persistent workgroup per slot; trajectories taken in turn.
__global__ void __launch_bounds__(kThreads) k_batch_small(const BSmall *__restrict__ small, int n_small,
                                                          const BBlock *__restrict__ blocks,
                                                          const float2 *__restrict__ mats, float2 *__restrict__ buf,
                                                          double *__restrict__ z0)
{
    extern __shared__ float2 lds[];
    for (int s = blockIdx.x; s < n_small; s += gridDim.x) {
        const BSmall tr = small[s];
        const uint32_t N = 1u << tr.n;
        for (uint32_t i = threadIdx.x; i < N; i += kThreads) lds[i] = make_float2(i == 0 ? 1.f : 0.f, 0.f);
        __syncthreads();
        for (int bi = 0; bi < tr.n_blocks; ++bi) {
            const BBlock b = blocks[tr.first_block + bi];
            const uint32_t groups = N >> b.k;
            for (uint32_t g = threadIdx.x; g < groups; g += kThreads) apply_group_k(lds, b, mats + b.mat_off, g);
            __syncthreads();
        }
        double acc = 0.0;
        for (uint32_t i = threadIdx.x; i < N; i += kThreads) {
            const float2 v = lds[i];
            const double p = double(v.x) * v.x + double(v.y) * v.y;
            acc += (i & 1) ? -p : p;
        }
        const double z = block_sum(acc);
        if (threadIdx.x == 0) z0[tr.out] = z;
        float2 *dst = buf + tr.state_off;
        for (uint32_t i = threadIdx.x; i < N; i += kThreads) dst[i] = lds[i];
        __syncthreads();
    }
}

__global__ void k_batch_zero(float2 *__restrict__ buf, uint64_t begin, uint64_t end)
{
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = begin + uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < end; i += stride)
        buf[i] = make_float2(0.f, 0.f);
}

__global__ void k_batch_one(const BLarge *__restrict__ large, int n_large, float2 *__restrict__ buf)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n_large) buf[large[t].state_off] = make_float2(1.f, 0.f);
}

// <Z_0> partial sums: one workgroup per chunk of one state (chunks start at
// even indices, so the parity of the local index is that of the state index).
__global__ void __launch_bounds__(kThreads) k_batch_z0_part(const BZUnit *__restrict__ units,
                                                            const float2 *__restrict__ buf,
                                                            double *__restrict__ partial)
{
    const BZUnit u = units[blockIdx.x];
    const float2 *st = buf + u.off;
    double acc = 0.0;
    for (uint32_t i = threadIdx.x; i < u.count; i += kThreads) {
        const float2 v = st[i];
        const double p = double(v.x) * v.x + double(v.y) * v.y;
        acc += (i & 1) ? -p : p;
    }
    const double z = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = z;
}

// Per trajectory: its partial sums in chunk order.
__global__ void k_batch_z0_final(const BLarge *__restrict__ large, int n_large, const double *__restrict__ partial,
                                 double *__restrict__ z0)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_large) return;
    const BLarge tr = large[t];
    double z = 0.0;
    for (int c = 0; c < tr.zcount; ++c) z += partial[tr.zfirst + c];
    z0[tr.out] = z;
}

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

struct sv_batch {
    int n_traj = 0;
    int max_k = 0;
    int tile_prec = dev::kTileOperandF32;  // arithmetic of the large trajectories' tile passes
    hipStream_t stream = nullptr;
    hipStream_t side = nullptr;  // fork stream for graph capture / overlap
    hipEvent_t fork = nullptr, join = nullptr;
    float2 *buf = nullptr;
    std::vector<int32_t> n_qubits;
    std::vector<uint64_t> state_off;  // complex elements
    // device tables
    DevBuf d_blocks, d_mats, d_small, d_large, d_z0;
    DevBuf d_passes, d_units, d_pool, d_zunits, d_partial;
    int n_small = 0, n_large = 0, small_max_n = 0, n_zunits = 0;
    uint64_t large_begin = 0, large_end = 0;
    std::vector<std::pair<size_t, int>> steps;  // per layer: (offset into units, count)
    PinBuf h_z0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~sv_batch()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (side) (void)hipStreamDestroy(side);
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
    }
};

namespace {

int check_desc(const sv_batch_desc *d)
{
    if (!d) return fail(SV_ERR_ARG, "NULL batch description");
    if (d->n_traj < 1) return fail(SV_ERR_ARG, "batch needs at least one trajectory");
    if (!d->n_qubits || !d->gate_offsets) return fail(SV_ERR_ARG, "NULL batch arrays");
    if (d->max_k != -1 && (d->max_k < 1 || d->max_k > SV_MAX_K)) return fail(SV_ERR_ARG, "max_k %d", d->max_k);
    if (d->precision != SV_PREC_FP32 && d->precision != SV_PREC_SPLIT_BF16 && d->precision != SV_PREC_SPLIT_FP16 &&
        d->precision != SV_PREC_SPLIT_BF16X3)
        return fail(SV_ERR_ARG, "batch precision %d (FP32, split BF16, split FP16 or split BF16X3)", d->precision);
    if (d->gate_offsets[0] != 0) return fail(SV_ERR_ARG, "gate_offsets[0] must be 0");
    for (int t = 0; t < d->n_traj; ++t) {
        const int n = d->n_qubits[t];
        if (n < 1 || n > 30) return fail(SV_ERR_ARG, "trajectory %d: n = %d outside 1..30", t, n);
        if (d->gate_offsets[t + 1] < d->gate_offsets[t]) return fail(SV_ERR_ARG, "gate_offsets decrease at %d", t);
        if (d->gate_offsets[t + 1] > d->gate_offsets[t] && !d->gates) return fail(SV_ERR_ARG, "NULL gates");
        for (int64_t g = d->gate_offsets[t]; g < d->gate_offsets[t + 1]; ++g) {
            int rc = check_gate_shape(d->gates[g]);
            if (!rc) rc = check_gate_qubits(d->gates[g], n);
            if (!rc && d->precision == SV_PREC_SPLIT_FP16) rc = check_fp16_gates(d->gates + g, 1);
            if (rc) return rc;
        }
    }
    return SV_OK;
}

size_t state_bytes(int n) { return al256((size_t(1) << n) * sizeof(float2)); }

// Fuse every trajectory with limit k and upload the work tables.
int build_schedule(sv_batch *b, const sv_batch_desc *d, int k)
{
    std::vector<BBlock> blocks;
    std::vector<float2> mats;
    std::vector<BSmall> small;
    std::vector<BLarge> large;
    std::vector<dev::TilePass> passes;
    std::vector<uint32_t> pool;                  // tile operands (pack_tile_operand), one per block
    std::vector<std::vector<int>> large_passes;  // per large trajectory: its pass indices
    std::vector<BZUnit> zunits;
    const CostTable cost = default_costs();
    const int max_sub = dev::tile_max_blocks(dev::kBatchTileBits, dev::kBatchTileWaves, b->tile_prec);
    for (int t = 0; t < d->n_traj; ++t) {
        const int n = d->n_qubits[t];
        const sv_gate *g = d->gates + d->gate_offsets[t];
        const int G = int(d->gate_offsets[t + 1] - d->gate_offsets[t]);
        int kk = k;
        for (int i = 0; i < G; ++i) kk = std::max(kk, g[i].k);
        kk = std::min(kk, n);
        if (n <= kSmallMaxN) {
            std::vector<Block> fb;
            if (int rc = fuse_gates(g, G, n, kk, SV_RULE_ENHANCED, cost, fb)) return rc;
            const int first = int(blocks.size());
            for (const Block &B : fb) {
                BBlock x;
                std::memset(&x, 0, sizeof x);
                x.state_off = b->state_off[t];
                x.n = n;
                x.k = B.k;
                for (int j = 0; j < B.k; ++j) x.q[j] = B.q[j];
                x.mat_off = int(mats.size());
                for (const cd &v : B.m) mats.push_back(make_float2(float(v.real()), float(v.imag())));
                blocks.push_back(x);
            }
            small.push_back({b->state_off[t], n, first, int(fb.size()), t});
            continue;
        }
        // tiled plan: groups of consecutive blocks of one pass, at most max_sub per launch
        std::vector<Block> fb;
        if (int rc = fuse_gates(g, G, n, std::min(kk, 4), SV_RULE_TILED, cost, fb, true, d->precision)) return rc;
        std::vector<int> mine;
        for (const auto &grp : tile_groups(fb, n)) {
            for (size_t c = 0; c < grp.size(); c += size_t(max_sub)) {
                const int cnt = int(std::min(grp.size() - c, size_t(max_sub)));
                std::vector<const Block *> bp;
                for (int i = 0; i < cnt; ++i) bp.push_back(&fb[grp[c + i]]);
                int sub_pos[dev::kMaxTileSubBlocks][4];
                std::vector<cd> m4;
                tile_pass_blocks(bp.data(), cnt, n, sub_pos, m4);
                dev::TilePass tp;
                std::memset(&tp, 0, sizeof tp);
                tp.state_off = b->state_off[t];
                tp.op_off = pool.size();
                if (dev::make_tile_args(cnt, sub_pos, n, dev::kBatchTileBits, dev::kBatchTileWaves, b->tile_prec,
                                       &tp.args) != hipSuccess)
                    return fail(SV_ERR_ARG, "trajectory %d: tile pass layout", t);
                pool.resize(pool.size() + size_t(cnt) * dev::kTileOperandWords);
                for (int i = 0; i < cnt; ++i)
                    dev::pack_tile_operand(m4.data() + 256 * i, b->tile_prec, pool.data() + tp.op_off + dev::kTileOperandWords * i);
                mine.push_back(int(passes.size()));
                passes.push_back(tp);
            }
        }
        BLarge L;
        L.state_off = b->state_off[t];
        L.n = n;
        L.out = t;
        L.zfirst = int(zunits.size());
        const uint64_t N = uint64_t(1) << n, chunk = uint64_t(1) << kZ0ChunkBits;
        for (uint64_t o = 0; o < N; o += chunk) zunits.push_back({b->state_off[t] + o, uint32_t(std::min(chunk, N - o)), 0});
        L.zcount = int(zunits.size()) - L.zfirst;
        large.push_back(L);
        large_passes.push_back(mine);
    }
    // layered launches: layer s holds pass s of every large trajectory, as
    // tile ranges (a quarter of the tiles of the largest states per unit)
    std::vector<dev::TileUnit> units;
    b->steps.clear();
    size_t layers = 0;
    for (auto &v : large_passes) layers = std::max(layers, v.size());
    for (size_t s = 0; s < layers; ++s) {
        const size_t off = units.size();
        for (auto &v : large_passes) {
            if (s >= v.size()) continue;
            const dev::TilePass &tp = passes[v[s]];
            const uint64_t nt = tp.args.n_tiles;
            const uint64_t per = std::max<uint64_t>(1, nt / 64);
            for (uint64_t t0 = 0; t0 < nt; t0 += per) units.push_back({v[s], 0, t0, std::min(nt, t0 + per)});
        }
        b->steps.push_back({off, int(units.size() - off)});
    }
    b->n_small = int(small.size());
    b->n_large = int(large.size());
    b->n_zunits = int(zunits.size());
    b->small_max_n = 0;
    for (auto &s : small) b->small_max_n = std::max(b->small_max_n, s.n);
    // large states are laid out after the small ones, contiguously
    b->large_begin = b->large_end = 0;
    if (!large.empty()) {
        b->large_begin = large.front().state_off;
        for (auto &l : large) {
            b->large_begin = std::min(b->large_begin, l.state_off);
            b->large_end = std::max(b->large_end, l.state_off + (uint64_t(1) << l.n));
        }
    }
    auto upload = [](DevBuf &dst, const void *src, size_t bytes) -> hipError_t {
        hipError_t e = dst.ensure(std::max(bytes, size_t(256)));
        if (e == hipSuccess && bytes) e = hipMemcpy(dst.p, src, bytes, hipMemcpyHostToDevice);
        return e;
    };
    SV_HIP(upload(b->d_blocks, blocks.data(), blocks.size() * sizeof(BBlock)));
    SV_HIP(upload(b->d_mats, mats.data(), mats.size() * sizeof(float2)));
    SV_HIP(upload(b->d_small, small.data(), small.size() * sizeof(BSmall)));
    SV_HIP(upload(b->d_large, large.data(), large.size() * sizeof(BLarge)));
    SV_HIP(upload(b->d_passes, passes.data(), passes.size() * sizeof(dev::TilePass)));
    SV_HIP(upload(b->d_units, units.data(), units.size() * sizeof(dev::TileUnit)));
    SV_HIP(upload(b->d_pool, pool.data(), pool.size() * sizeof(uint32_t)));
    SV_HIP(upload(b->d_zunits, zunits.data(), zunits.size() * sizeof(BZUnit)));
    SV_HIP(b->d_partial.ensure(std::max<size_t>(zunits.size(), 1) * sizeof(double)));
    b->max_k = k;
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    return SV_OK;
}

// Enqueue one full run: small kernel on `side`, large chain on `main`.
int enqueue_run(sv_batch *b, hipStream_t main, hipStream_t side)
{
    double *z0 = static_cast<double *>(b->d_z0.p);
    const auto *blocks = static_cast<const BBlock *>(b->d_blocks.p);
    const auto *mats = static_cast<const float2 *>(b->d_mats.p);
    SV_HIP(hipEventRecord(b->fork, main));
    SV_HIP(hipStreamWaitEvent(side, b->fork, 0));
    if (b->n_small) {
        LaunchTimer t(stat_class(FAM_BATCH, 1), side);
        const unsigned grid = unsigned(std::min(b->n_small, 2048));
        const size_t lds = size_t(sizeof(float2)) << b->small_max_n;
        hipLaunchKernelGGL(k_batch_small, dim3(grid), dim3(kThreads), lds, side,
                           static_cast<const BSmall *>(b->d_small.p), b->n_small, blocks, mats, b->buf, z0);
        SV_HIP(hipGetLastError());
    }
    if (b->n_large) {
        {
            LaunchTimer t(stat_class(FAM_BATCH, 2), main);
            const uint64_t cnt = b->large_end - b->large_begin;
            const unsigned grid = unsigned(std::min<uint64_t>((cnt + 255) / 256, 16384));
            hipLaunchKernelGGL(k_batch_zero, dim3(grid), dim3(256), 0, main, b->buf, b->large_begin, b->large_end);
            hipLaunchKernelGGL(k_batch_one, dim3((b->n_large + 255) / 256), dim3(256), 0, main,
                               static_cast<const BLarge *>(b->d_large.p), b->n_large, b->buf);
            SV_HIP(hipGetLastError());
        }
        const auto *units = static_cast<const dev::TileUnit *>(b->d_units.p);
        const auto *passes = static_cast<const dev::TilePass *>(b->d_passes.p);
        const auto *pool = static_cast<const uint32_t *>(b->d_pool.p);
        for (const auto &st : b->steps) {
            LaunchTimer t(stat_class(FAM_BATCH, 3), main);
            SV_HIP(dev::launch_tile_batch(units + st.first, st.second, passes, pool, b->buf, main, b->tile_prec));
        }
        LaunchTimer t(stat_class(FAM_BATCH, 4), main);
        double *partial = static_cast<double *>(b->d_partial.p);
        hipLaunchKernelGGL(k_batch_z0_part, dim3(b->n_zunits), dim3(kThreads), 0, main,
                           static_cast<const BZUnit *>(b->d_zunits.p), b->buf, partial);
        hipLaunchKernelGGL(k_batch_z0_final, dim3((b->n_large + 255) / 256), dim3(256), 0, main,
                           static_cast<const BLarge *>(b->d_large.p), b->n_large, partial, z0);
        SV_HIP(hipGetLastError());
    }
    SV_HIP(hipEventRecord(b->join, side));
    SV_HIP(hipStreamWaitEvent(main, b->join, 0));
    return SV_OK;
}

int run_once(sv_batch *b, int use_graph)
{
    if (!use_graph) return enqueue_run(b, b->stream, b->side);
    if (!b->exec) {
        // capture on a private stream (capture is not allowed on the null stream)
        hipStream_t cs;
        SV_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        SV_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        timing_suspend(true);
        int rc = enqueue_run(b, cs, b->side);
        timing_suspend(false);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(cs, &g);
        (void)hipStreamDestroy(cs);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return fail(SV_ERR_HIP, "batch graph capture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        b->graph = g;
        if (e != hipSuccess) return fail(SV_ERR_HIP, "batch graph instantiate: %s", hipGetErrorString(e));
    }
    SV_HIP(hipGraphLaunch(b->exec, b->stream));
    return SV_OK;
}

}  // namespace

extern "C" int sv_batch_required_bytes(const sv_batch_desc *d, size_t *out)
{
    clear_error();
    if (!out) return fail(SV_ERR_ARG, "NULL out");
    if (int rc = check_desc(d)) return rc;
    size_t total = 0;
    for (int t = 0; t < d->n_traj; ++t) total += state_bytes(d->n_qubits[t]);
    *out = total;
    return SV_OK;
}

extern "C" int sv_batch_create(const sv_batch_desc *d, void *dev_buf, size_t bytes, void *hip_stream,
                               sv_batch **out)
{
    clear_error();
    if (!out) return fail(SV_ERR_ARG, "NULL out");
    *out = nullptr;
    size_t need = 0;
    if (int rc = sv_batch_required_bytes(d, &need)) return rc;
    if (!dev_buf) return fail(SV_ERR_ARG, "NULL device buffer");
    if (bytes < need) return fail(SV_ERR_SIZE, "batch needs %zu bytes, got %zu", need, bytes);
    if (reinterpret_cast<uintptr_t>(dev_buf) % 256) return fail(SV_ERR_ARG, "device buffer not 256-byte aligned");
    std::unique_ptr<sv_batch> b(new sv_batch);
    b->n_traj = d->n_traj;
    b->tile_prec = tile_operand_prec(tile_path(d->precision));
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->buf = static_cast<float2 *>(dev_buf);
    b->n_qubits.assign(d->n_qubits, d->n_qubits + d->n_traj);
    // small states first, then large ones (contiguous), each 256-byte aligned
    b->state_off.assign(d->n_traj, 0);
    size_t off = 0;
    for (int pass = 0; pass < 2; ++pass)
        for (int t = 0; t < d->n_traj; ++t) {
            const bool small = d->n_qubits[t] <= kSmallMaxN;
            if (small != (pass == 0)) continue;
            b->state_off[t] = off / sizeof(float2);
            off += state_bytes(d->n_qubits[t]);
        }
    SV_HIP(hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking));
    SV_HIP(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
    SV_HIP(hipEventCreateWithFlags(&b->join, hipEventDisableTiming));
    SV_HIP(b->d_z0.ensure(sizeof(double) * d->n_traj));
    SV_HIP(b->h_z0.ensure(sizeof(double) * d->n_traj));
    if (d->max_k != -1) {
        if (int rc = build_schedule(b.get(), d, d->max_k)) return rc;
    } else {
        // autotune the fusion limit on this batch
        hipEvent_t e0, e1;
        SV_HIP(hipEventCreate(&e0));
        SV_HIP(hipEventCreate(&e1));
        double best = 1e300;
        int best_k = 3;
        timing_suspend(true);
        for (int k = 2; k <= 4; ++k) {
            int rc = build_schedule(b.get(), d, k);
            if (!rc) rc = enqueue_run(b.get(), b->stream, b->side);  // warm-up
            if (!rc && hipEventRecord(e0, b->stream) != hipSuccess) rc = fail(SV_ERR_HIP, "event record");
            if (!rc) rc = enqueue_run(b.get(), b->stream, b->side);
            if (!rc && hipEventRecord(e1, b->stream) != hipSuccess) rc = fail(SV_ERR_HIP, "event record");
            float ms = 0;
            if (!rc && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = fail(SV_ERR_HIP, "batch autotune timing");
            if (rc) {
                timing_suspend(false);
                return rc;
            }
            if (ms < best) {
                best = ms;
                best_k = k;
            }
        }
        timing_suspend(false);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (int rc = build_schedule(b.get(), d, best_k)) return rc;
    }
    *out = b.release();
    return SV_OK;
}

extern "C" int sv_batch_run(sv_batch *b, int use_graph, double *z0_out)
{
    clear_error();
    if (!b || !z0_out) return fail(SV_ERR_ARG, "NULL argument");
    if (int rc = run_once(b, use_graph)) return rc;
    SV_HIP(hipMemcpyAsync(b->h_z0.p, b->d_z0.p, sizeof(double) * b->n_traj, hipMemcpyDeviceToHost, b->stream));
    SV_HIP(hipStreamSynchronize(b->stream));
    std::memcpy(z0_out, b->h_z0.p, sizeof(double) * b->n_traj);
    return SV_OK;
}

extern "C" int sv_batch_read(sv_batch *b, int t, uint64_t first, uint64_t count, void *host)
{
    clear_error();
    if (!b) return fail(SV_ERR_ARG, "NULL batch");
    if (t < 0 || t >= b->n_traj) return fail(SV_ERR_ARG, "trajectory %d out of range", t);
    const uint64_t N = uint64_t(1) << b->n_qubits[t];
    if (first > N || count > N - first) return fail(SV_ERR_ARG, "range outside the state");
    if (count && !host) return fail(SV_ERR_ARG, "NULL host buffer");
    if (count)
        SV_HIP(hipMemcpyAsync(host, b->buf + b->state_off[t] + first, count * sizeof(float2), hipMemcpyDeviceToHost,
                              b->stream));
    SV_HIP(hipStreamSynchronize(b->stream));
    return SV_OK;
}

extern "C" int sv_batch_free(sv_batch *b)
{
    if (!b) return SV_OK;
    (void)hipStreamSynchronize(b->stream);
    (void)hipStreamSynchronize(b->side);
    delete b;
    return SV_OK;
}
