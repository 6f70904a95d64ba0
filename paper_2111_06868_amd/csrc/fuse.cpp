// Greedy gate fusion (host only, no HIP calls).
//
// Paper, Circuit utilities section: compress(circuit, max_n_qubits) groups the
// gates into blocks of at most max_n_qubits qubits, each applied as one dense
// matrix (to_matrix_gate).  Its printed example (CPHASE on all pairs of five
// qubits, max_n_qubits = 3 -> blocks (0,1,2), (0,3,4), (1,3,4), (2,3,4)) fixes
// the rule for gates that meet an existing block: a gate joins the LAST block
// that shares a qubit with it when the union fits, else it opens a new block.
// That placement is legal because every later block is disjoint from the gate.
//
// The enhanced rule keeps that first pass and adds two cost-aware steps:
//   - a gate that cannot join the last intersecting block may join any later
//     block (all of them are disjoint from it) when the cost table says the
//     grown block is cheaper than a block of its own;
//   - afterwards, block j is merged into an earlier block i when every block
//     between them is disjoint from j (so j commutes next to i) and the cost
//     of the union is lower than the two costs together.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>

#include "common.h"

namespace sv {

CostTable default_costs()
{
    // One state pass per block is the dominant cost on an HBM-bound path;
    // larger blocks cost somewhat more arithmetic.  Relative units.
    CostTable t;
    t.valid = true;
    const double c[SV_MAX_K + 1] = {0.0, 1.0, 1.0, 1.0, 1.02, 1.1, 1.6};
    std::memcpy(t.ms, c, sizeof c);
    // a tile pass is one state pass plus in-LDS work per 4-qubit block
    const double tl[5] = {0.0, 1.1, 1.15, 1.3, 1.5};
    std::memcpy(t.tile, tl, sizeof tl);
    return t;
}

static std::mutex g_cost_mu;
static std::map<std::pair<int, int>, CostTable> g_costs;

CostTable lookup_costs(int n, int precision, bool *found)
{
    std::lock_guard<std::mutex> lk(g_cost_mu);
    auto it = g_costs.find({n, precision});
    if (it != g_costs.end()) {
        if (found) *found = true;
        return it->second;
    }
    if (found) *found = false;
    return default_costs();
}

void store_costs(int n, int precision, const double *ms, const double *tile)
{
    CostTable t = default_costs();
    t.valid = true;
    for (int k = 0; k <= SV_MAX_K; ++k) t.ms[k] = ms[k];
    if (tile) {
        for (int s = 0; s <= 4; ++s) t.tile[s] = tile[s];
    } else {
        // untimed tile passes: scale the defaults by the measured 4-qubit block cost
        for (int s = 1; s <= 4; ++s) t.tile[s] *= ms[4] / default_costs().ms[4];
    }
    std::lock_guard<std::mutex> lk(g_cost_mu);
    g_costs[{n, precision}] = t;
}

namespace {

struct WBlock {
    uint64_t mask = 0;  // qubit positions as a bit set
    std::vector<int> members;
};

inline int popc(uint64_t x) { return __builtin_popcountll(x); }

uint64_t gate_mask(const sv_gate &g)
{
    uint64_t m = 0;
    for (int j = 0; j < g.k; ++j) m |= uint64_t(1) << g.q[j];
    return m;
}

}  // namespace

double plan_cost(const std::vector<Block> &blocks, const CostTable &cost)
{
    double s = 0;
    for (auto &b : blocks) s += cost.ms[b.k];
    return s;
}

// Apply a canonical gate matrix (on block-local bits lb[0..kg-1], ascending)
// to every column of the D x D canonical block matrix U (in place).  Plain
// real arithmetic on (re, im) pairs: std::complex multiplication carries
// inf/nan recovery that dominates the cost of fusing large blocks.
static void apply_to_columns(std::vector<cd> &Uc, int kb, const std::vector<cd> &Gc, int kg, const int *lb)
{
    const int D = 1 << kb, Dg = 1 << kg;
    double *U = reinterpret_cast<double *>(Uc.data());
    const double *G = reinterpret_cast<const double *>(Gc.data());
    int tmask = 0;
    for (int j = 0; j < kg; ++j) tmask |= 1 << lb[j];
    int off[1 << SV_MAX_K];
    for (int m = 0; m < Dg; ++m) {
        off[m] = 0;
        for (int j = 0; j < kg; ++j)
            if ((m >> j) & 1) off[m] |= 1 << lb[j];
    }
    double vr[1 << SV_MAX_K], vi[1 << SV_MAX_K];
    for (int base = 0; base < D; ++base) {
        if (base & tmask) continue;
        for (int col = 0; col < D; ++col) {
            for (int m = 0; m < Dg; ++m) {
                const size_t e = 2 * (size_t(base | off[m]) * D + col);
                vr[m] = U[e];
                vi[m] = U[e + 1];
            }
            for (int m = 0; m < Dg; ++m) {
                double ar = 0, ai = 0;
                const double *g = G + 2 * size_t(m) * Dg;
                for (int mp = 0; mp < Dg; ++mp) {
                    ar += g[2 * mp] * vr[mp] - g[2 * mp + 1] * vi[mp];
                    ai += g[2 * mp] * vi[mp] + g[2 * mp + 1] * vr[mp];
                }
                const size_t e = 2 * (size_t(base | off[m]) * D + col);
                U[e] = ar;
                U[e + 1] = ai;
            }
        }
    }
}

void block_matrix(const sv_gate *g, Block &b)
{
    const int D = 1 << b.k;
    b.m.assign(size_t(D) * D, cd(0));
    for (int i = 0; i < D; ++i) b.m[size_t(i) * D + i] = 1;
    std::vector<cd> G;
    for (int gi : b.members) {
        int sq[SV_MAX_K];
        gate_matrix_canonical(g[gi], G, sq);
        int lb[SV_MAX_K];
        for (int j = 0; j < g[gi].k; ++j) {
            int r = 0;
            while (b.q[r] != sq[j]) ++r;
            lb[j] = r;
        }
        apply_to_columns(b.m, b.k, G, g[gi].k, lb);
    }
}

int fuse_gates(const sv_gate *g, int G, int n, int max_k, int rule, const CostTable &cost,
               std::vector<Block> &blocks, bool with_matrices)
{
    (void)n;
    if (max_k < 1 || max_k > SV_MAX_K) return fail(SV_ERR_ARG, "max_k %d outside 1..%d", max_k, SV_MAX_K);
    if (rule == SV_RULE_TILED) {  // blocks for tile passes: the enhanced rule, at most 4 qubits
        rule = SV_RULE_ENHANCED;
        max_k = max_k < 4 ? max_k : 4;
    }
    if (rule != SV_RULE_PAPER && rule != SV_RULE_ENHANCED && rule != SV_RULE_NONE)
        return fail(SV_ERR_ARG, "unknown fusion rule %d", rule);
    std::vector<WBlock> wb;
    wb.reserve(G);
    for (int gi = 0; gi < G; ++gi) {
        const uint64_t gm = gate_mask(g[gi]);
        if (g[gi].k > max_k && rule != SV_RULE_NONE)
            return fail(SV_ERR_ARG, "gate %d acts on %d qubits, more than max_k=%d", gi, g[gi].k, max_k);
        if (rule == SV_RULE_NONE) {
            wb.push_back({gm, {gi}});
            continue;
        }
        int last = -1;
        for (int b = int(wb.size()) - 1; b >= 0; --b)
            if (wb[b].mask & gm) { last = b; break; }
        if (last >= 0 && popc(wb[last].mask | gm) <= max_k) {
            wb[last].mask |= gm;
            wb[last].members.push_back(gi);
            continue;
        }
        if (rule == SV_RULE_ENHANCED) {
            int best = -1;
            double best_gain = 1e-12;
            for (int b = last + 1; b < int(wb.size()); ++b) {
                int ku = popc(wb[b].mask | gm);
                if (ku > max_k) continue;
                double gain = cost.ms[popc(wb[b].mask)] + cost.ms[popc(gm)] - cost.ms[ku];
                if (gain > best_gain) { best_gain = gain; best = b; }
            }
            if (best >= 0) {
                wb[best].mask |= gm;
                wb[best].members.push_back(gi);
                continue;
            }
        }
        wb.push_back({gm, {gi}});
    }
    if (rule == SV_RULE_ENHANCED) {
        bool changed = true;
        while (changed) {
            changed = false;
            for (int j = 1; j < int(wb.size()); ++j) {
                for (int i = j - 1; i >= 0; --i) {
                    const uint64_t u = wb[i].mask | wb[j].mask;
                    const int ku = popc(u);
                    if (ku <= max_k &&
                        cost.ms[ku] < cost.ms[popc(wb[i].mask)] + cost.ms[popc(wb[j].mask)] - 1e-12) {
                        wb[i].mask = u;
                        wb[i].members.insert(wb[i].members.end(), wb[j].members.begin(), wb[j].members.end());
                        wb.erase(wb.begin() + j);
                        changed = true;
                        --j;
                        break;
                    }
                    if (wb[i].mask & wb[j].mask) break;  // j cannot move past block i
                }
            }
        }
    }
    blocks.clear();
    blocks.resize(wb.size());
    size_t work = 0;
    for (size_t b = 0; b < wb.size(); ++b) {
        Block &B = blocks[b];
        B.k = 0;
        for (int p = 0; p < 64; ++p)
            if ((wb[b].mask >> p) & 1) B.q[B.k++] = p;
        B.members = wb[b].members;
        work += B.members.size() << (2 * B.k);
    }
    if (!with_matrices) return SV_OK;
    // block matrices are independent: spread large jobs over host threads
    const unsigned hw = std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
    const unsigned nt = work > (size_t(1) << 18) ? std::min<unsigned>(hw, unsigned(blocks.size())) : 1u;
    std::atomic<size_t> next(0);
    auto worker = [&]() {
        for (size_t b; (b = next.fetch_add(1)) < blocks.size();) block_matrix(g, blocks[b]);
    };
    std::vector<std::thread> pool;
    for (unsigned t = 1; t < nt; ++t) pool.emplace_back(worker);
    worker();
    for (auto &th : pool) th.join();
    return SV_OK;
}

std::vector<std::vector<size_t>> tile_groups(const std::vector<Block> &blocks, int n)
{
    // Greedy, commutation-aware: a group starts at the first block not yet
    // applied and takes later blocks of <= 4 qubits while the union stays
    // within 8 positions; a later block may join only if it is disjoint from
    // every block it jumps over (so it commutes past them).
    constexpr int kMaxUnion = 8, kMaxBlocks = 4, kMinQubits = 14;
    auto mask_of = [](const Block &b) {
        uint64_t m = 0;
        for (int j = 0; j < b.k; ++j) m |= uint64_t(1) << b.q[j];
        return m;
    };
    std::vector<std::vector<size_t>> out;
    std::vector<char> done(blocks.size(), 0);
    for (size_t i = 0; i < blocks.size(); ++i) {
        if (done[i]) continue;
        std::vector<size_t> grp = {i};
        uint64_t um = mask_of(blocks[i]);
        if (blocks[i].k <= 4 && n >= kMinQubits) {
            uint64_t skipped = 0;
            for (size_t j = i + 1; j < blocks.size() && int(grp.size()) < kMaxBlocks; ++j) {
                if (done[j]) continue;
                const uint64_t m = mask_of(blocks[j]);
                if (!(m & skipped) && blocks[j].k <= 4 && popc(um | m) <= kMaxUnion) {
                    um |= m;
                    grp.push_back(j);
                } else {
                    skipped |= m;
                }
            }
        }
        if (grp.size() < 2) grp.resize(1);
        for (size_t b : grp) done[b] = 1;
        out.push_back(std::move(grp));
    }
    return out;
}

double tiled_plan_cost(const std::vector<Block> &blocks, int n, const CostTable &cost)
{
    double c = 0;
    for (const auto &grp : tile_groups(blocks, n))
        c += grp.size() == 1 ? cost.ms[blocks[grp[0]].k] : cost.tile[grp.size()];
    return c;
}

}  // namespace sv
