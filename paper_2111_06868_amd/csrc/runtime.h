// Runtime pieces shared by the API translation units: state handle, device
// buffers, launch timing, kernel-path selection and tuning knobs.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "kernels.h"

#define SV_HIP(expr)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return sv::fail(SV_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

namespace sv {

// Growable device buffer (hipMalloc; freed on destruction).
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t bytes);
    void release();
    ~DevBuf() { release(); }
};

// Growable pinned host buffer.
struct PinBuf {
    void *p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t bytes);
    void release();
    ~PinBuf() { release(); }
};

// Kernel families for timing (class = 100 * family + k, see stat_class).
enum Family {
    FAM_REG = 1,
    FAM_GENERIC = 2,
    FAM_MFMA32 = 3,
    FAM_SPLIT_BF16 = 4,
    FAM_SPLIT_FP16 = 5,
    FAM_REDUCE = 6,
    FAM_ADJOINT = 7,
    FAM_BATCH = 8,
    FAM_TILE = 9,
    FAM_TILE_BF16 = 10,
    FAM_TILE_FP16 = 11,
    FAM_TILE_BF16X3 = 12,
};

// Statistics class of a launch: 100 * family + k (k = block size, or the
// number of blocks of a tile pass).
inline int stat_class(int family, int k) { return 100 * family + k; }

// RAII: brackets one launch with HIP events on `st` when timing is enabled.
class LaunchTimer {
  public:
    LaunchTimer(int cls, hipStream_t st);
    ~LaunchTimer();
    LaunchTimer(const LaunchTimer &) = delete;
    LaunchTimer &operator=(const LaunchTimer &) = delete;

  private:
    int cls_;
    hipStream_t st_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
};
// Suspend timing (inside graph capture).
void timing_suspend(bool on);

// Kernel paths for a block.
enum Path {
    PATH_REG,
    PATH_GENERIC,
    PATH_MFMA32,
    PATH_SPLIT_BF16,
    PATH_SPLIT_FP16,
    PATH_TILE,
    PATH_TILE_BF16,
    PATH_TILE_FP16,
    PATH_TILE_BF16X3
};

// Tile passes: PATH_TILE, PATH_TILE_BF16, PATH_TILE_FP16, PATH_TILE_BF16X3.
inline bool is_tile_path(int p)
{
    return p == PATH_TILE || p == PATH_TILE_BF16 || p == PATH_TILE_FP16 || p == PATH_TILE_BF16X3;
}

struct Tuning {
    int reg_grid_cap[SV_MAX_K + 1];   // 0 = one thread per group
    int mfma_tc_log[SV_MAX_K + 1];    // log2 columns per tile
    int mfma_grid_cap[SV_MAX_K + 1];
    int split_tc_log[SV_MAX_K + 1];
    bool k4_reg;                      // FP32: k = 4 via the register kernel
    int tile_grid_cap;                // workgroups per resident slot set (one per CU)
    int tile_bits;                    // 13 (64 KiB LDS tiles) or 14 (128 KiB)
    int tile_waves;                   // waves per tile workgroup (4 or 8)
};
Tuning &tuning();
Path choose_path(int dtype, int precision, int k, const int *sorted_q, int n);
int path_family(Path p);

// One block (or, for a tile path, a group of 4-qubit blocks) prepared for launch.
struct Launch {
    Path path;
    int k;                 // tile paths: number of blocks in the group
    int q[SV_MAX_K];
    std::vector<cd> m;     // canonical matrix; tile paths: k matrices of 16 x 16
    int sub_pos[dev::kMaxTileSubBlocks][4] = {};  // tile paths: each block's positions
    size_t arena_off = 0;  // byte offset of device operands (other paths)
    size_t arena_off2 = 0; // second and third operands (split parts 1 and 2)
    size_t arena_off3 = 0;
    size_t norm_off = 0;   // split-FP16 tile paths: byte offset of the run's norm partials
    int64_t basis = -1;    // tile paths, >= 0: the launch's first chunk starts the state from |basis>
};
// Doubles the norm partials of a run's split-FP16 tile passes may take (one
// per workgroup of the first such pass).
constexpr int kTileNormSlots = 4096;

// Pack the device operands of `launches` into `stage` (host) and return the
// total byte count; offsets are written into the launches.
size_t pack_operands(std::vector<Launch> &launches, int dtype, PinBuf &stage);
// Positions (4 per block, ascending) and padded 16 x 16 canonical matrices of
// a tile pass made of `count` blocks of <= 4 qubits: a smaller block is
// padded with the lowest positions of the pass's union (itself completed to
// at least 4 positions with the lowest free ones).
void tile_pass_blocks(const Block *const *blocks, int count, int n, int (*sub_pos)[4], std::vector<cd> &mats);
// Group consecutive blocks into tile passes (see tile.hip); blocks that do not
// join a group keep their own launch.
void group_tile_passes(const std::vector<Block> &blocks, int n, int precision, std::vector<Launch> &out);
// The tile path of a precision (FP32, split BF16, split FP16) and the operand
// format of a tile path.
Path tile_path(int precision);
int tile_operand_prec(int path);
// Enqueue the launches on `st` with device operands at `arena`.
int enqueue(const std::vector<Launch> &launches, int dtype, void *psi, int n, const void *arena,
            hipStream_t st);
// psi2 (optional): a second state that receives every launch too (one
// launch covering both where the kernel supports it).
int enqueue(const Launch *first, size_t count, int dtype, void *psi, int n, const void *arena, hipStream_t st,
            void *psi2 = nullptr);

// Install the autotuned cost tables and launch shapes saved in the tuning
// cache file `path` for the architecture of `device` (see sv_autotune).
int load_tuning(const char *path, int device, int *loaded);

// Pauli sums: validation (terms, masks below bit n, finite coefficients),
// and the device tables (terms grouped by x mask) laid out in host memory h
// for a copy to device address d: their byte size, and the fill, which also
// points P at d.
int check_pauli(const sv_pauli_sum *H, int n);
size_t pauli_table_bytes(const sv_pauli_sum *H);
void pauli_table_fill(const sv_pauli_sum *H, char *h, const char *d, dev::PauliDev &P);

}  // namespace sv

struct sv_state {
    int n = 0;
    int dtype = SV_C64;
    void *buf = nullptr;
    size_t bytes = 0;
    bool owns = false;
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;
    int device = 0;
    sv::DevBuf red;        // reduction partials + result
    sv::PinBuf red_host;   // pinned result readback
    sv::DevBuf arena;      // device operands (matrices, Pauli tables)
    sv::PinBuf stage;      // pinned staging of the operands
    hipEvent_t arena_free = nullptr;  // recorded after the last launch reading the arena
    hipGraphExec_t graph_exec = nullptr;  // last instantiated launch graph (use_graph runs)
    int64_t graph_launches = 0, graph_updates = 0;  // graph runs, and those that reused graph_exec
    sv::DevBuf grad;       // adjoint partials
};
