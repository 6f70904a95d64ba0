// Streaming read + write pass over a state at a chosen HBM layout: the
// achievable rate of one state pass, against which the tile passes' rate is
// judged.  Each workgroup moves tiles of 2^14 complex64 amplitudes (128 KiB)
// spanned by 14 given positions (position 0 among them), exactly as a tile
// pass with those tile positions copies its tiles, but with no LDS and no
// block work: 16-byte loads of the next tile are issued before the stores of
// the current one.  Every value is written back where it was read, so the
// state is unchanged.
#include <hip/hip_runtime.h>

#include "runtime.h"

namespace {

typedef float vf4 __attribute__((ext_vector_type(4)));

constexpr int kTileUnitBits = 13;  // 16-byte units (amplitude pairs) per tile, log2
constexpr int kThreads = 1024;
constexpr int kPerThread = (1 << kTileUnitBits) / kThreads;

struct StreamArgs {
    uint64_t n_tiles;
    int ubit[kTileUnitBits];                // tile unit bit -> unit bit of the state
    int ext_bit[SV_MAX_QUBITS_C64];         // unit bits outside the tile, ascending
    int n_ext;
};

__device__ __forceinline__ uint64_t tile_base(uint64_t T, const StreamArgs &a)
{
    uint64_t x = 0;
    for (int i = 0; i < a.n_ext; ++i) x |= ((T >> i) & 1) << a.ext_bit[i];
    return x;
}

__global__ void __launch_bounds__(kThreads) k_stream_rw(vf4 *__restrict__ psi, const StreamArgs a)
{
    const uint32_t tid = threadIdx.x;
    uint64_t off[kPerThread];
#pragma unroll
    for (int i = 0; i < kPerThread; ++i) {
        const uint32_t t = tid + i * kThreads;
        uint64_t g = 0;
#pragma unroll
        for (int b = 0; b < kTileUnitBits; ++b)
            if ((t >> b) & 1) g |= uint64_t(1) << a.ubit[b];
        off[i] = g;
    }
    uint64_t T = blockIdx.x;
    if (T >= a.n_tiles) return;
    vf4 cur[kPerThread], nxt[kPerThread];
    uint64_t base = tile_base(T, a);
#pragma unroll
    for (int i = 0; i < kPerThread; ++i) cur[i] = psi[base + off[i]];
    for (; T < a.n_tiles; T += gridDim.x) {
        const uint64_t Tn = T + gridDim.x;
        const uint64_t nbase = Tn < a.n_tiles ? tile_base(Tn, a) : 0;
        if (Tn < a.n_tiles) {
#pragma unroll
            for (int i = 0; i < kPerThread; ++i) nxt[i] = psi[nbase + off[i]];
        }
#pragma unroll
        for (int i = 0; i < kPerThread; ++i) psi[base + off[i]] = cur[i];
#pragma unroll
        for (int i = 0; i < kPerThread; ++i) cur[i] = nxt[i];
        base = nbase;
    }
}

}  // namespace

// Mean device milliseconds of `reps` passes (HIP events on the state's
// stream).  Synchronises.
extern "C" int sv_stream_probe(sv_state *s, uint64_t tile_positions, int reps, double *ms_per_pass)
{
    sv::clear_error();
    if (!s || !ms_per_pass) return sv::fail(SV_ERR_ARG, "NULL argument");
    if (s->dtype != SV_C64 || s->n < 14) return sv::fail(SV_ERR_ARG, "needs a complex64 state of >= 14 qubits");
    if (s->n < 64 && (tile_positions >> s->n))
        return sv::fail(SV_ERR_QUBIT, "tile positions beyond qubit %d", s->n - 1);
    if (__builtin_popcountll(tile_positions) != 14 || !(tile_positions & 1))
        return sv::fail(SV_ERR_ARG, "the tile needs 14 positions, position 0 among them");
    if (reps < 1 || reps > 1000) return sv::fail(SV_ERR_ARG, "reps = %d outside 1..1000", reps);
    SV_HIP(hipSetDevice(s->device));
    // unit bit u is position u + 1 (position 0 lies inside each 16-byte unit)
    StreamArgs a{};
    int b = 0;
    for (int p = 1; p < s->n; ++p) {
        if ((tile_positions >> p) & 1) a.ubit[b++] = p - 1;
        else a.ext_bit[a.n_ext++] = p - 1;
    }
    a.n_tiles = uint64_t(1) << a.n_ext;
    const unsigned grid = unsigned(a.n_tiles < 256 ? a.n_tiles : 256);  // one workgroup per compute unit
    hipEvent_t e0, e1;
    SV_HIP(hipEventCreate(&e0));
    SV_HIP(hipEventCreate(&e1));
    vf4 *psi = static_cast<vf4 *>(s->buf);
    hipError_t e = hipEventRecord(e0, s->stream);
    for (int i = 0; i < reps && e == hipSuccess; ++i) {
        hipLaunchKernelGGL(k_stream_rw, dim3(grid), dim3(kThreads), 0, s->stream, psi, a);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, s->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return sv::fail(SV_ERR_HIP, "stream probe: %s", hipGetErrorString(e));
    *ms_per_pass = double(ms) / reps;
    return SV_OK;
}
