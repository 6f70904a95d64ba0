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
// The enhanced rule builds two candidate plans and keeps the cheaper one
// under the cost table:
//   - the paper's pass plus two cost-aware steps: a gate that cannot join
//     the last intersecting block may join any later block (all of them are
//     disjoint from it) when the grown block is cheaper than a block of its
//     own, and block j is merged into an earlier block i when every block
//     between them is disjoint from j (so j commutes next to i) and the union
//     costs less than the two blocks;
//   - frontier grouping (frontier_groups): gates leave in any order that
//     keeps each qubit's gate sequence, and a block grows by the ready gate
//     that adds the fewest new positions.
// The tiled rule applies frontier grouping twice: passes whose positions
// form a tile of runs no shorter than those of a tile_union_limit()-position
// union (tile_union_fits), then blocks of at most 4 qubits inside each pass,
// which a tile kernel applies in one read and one write of the state.
#include <algorithm>
#include <atomic>
#include <cstdlib>
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
    // a tile pass is one state pass plus in-LDS work per 4-qubit block; one
    // block in a tile pass costs a little less than alone (the tile's HBM
    // copy runs at a higher rate than the dense kernels' strided access)
    t.tile[0] = 0;
    for (int s = 1; s <= kTilePassMaxBlocks; ++s) t.tile[s] = 0.9 + 0.07 * s;
    return t;
}

static int g_tile_union = [] {
    int u = 10;
    if (const char *e = std::getenv("SV_TILE_UNION")) u = std::atoi(e);
    return std::min(std::max(u, 8), kTilePassMaxUnion);
}();

int tile_union_limit() { return g_tile_union; }
void set_tile_union_limit(int u) { g_tile_union = std::min(std::max(u, 8), kTilePassMaxUnion); }

int tile_run_bits(uint64_t U, int tile_bits)
{
    uint64_t t = U;
    for (int p = 0; p < 64 && __builtin_popcountll(t) < tile_bits; ++p) t |= uint64_t(1) << p;
    int r = 0;
    while (r < 64 && ((t >> r) & 1)) ++r;
    return r;
}

bool tile_union_fits(uint64_t U, int n, int tile_bits, int limit)
{
    // a union of u <= limit positions leaves tile_bits - u fillers, and the
    // lowest positions 0 .. tile_bits - u - 1 are then all in the tile
    const int u = __builtin_popcountll(U);
    if (u <= limit) return true;
    return n >= tile_bits && u <= tile_bits && tile_run_bits(U, tile_bits) >= tile_bits - limit;
}

static std::mutex g_cost_mu;
static std::map<std::pair<int, int>, CostTable> g_costs;
static std::atomic<uint64_t> g_cost_version(1);

uint64_t cost_version() { return g_cost_version.load(); }

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
        for (int s = 0; s <= kTilePassMaxBlocks; ++s) t.tile[s] = tile[s];
    } else {
        // untimed tile passes: scale the defaults by the measured 4-qubit block cost
        for (int s = 1; s <= kTilePassMaxBlocks; ++s) t.tile[s] *= ms[4] / default_costs().ms[4];
    }
    std::lock_guard<std::mutex> lk(g_cost_mu);
    g_costs[{n, precision}] = t;
    ++g_cost_version;
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

// Frontier grouping of the gates idx[0..] (a sequence in which every
// qubit's gates already appear in circuit order).  Gates leave in an order
// that keeps each qubit's sequence, so the product of the groups, in order,
// equals the product of the gates.  A group starts with no positions; it takes
// every ready gate (first unapplied gate on each of its qubits) whose
// positions it already covers, and otherwise widens by the ready gate that
// adds the fewest positions (the earliest on ties) while it stays within
// what `fits` accepts (a predicate on position sets).  Members are listed in
// the order they are applied.  `fits` must accept every gate's own positions.
class Frontier {
  public:
    Frontier(const sv_gate *g, const std::vector<int> &idx) : idx_(idx), mask_(idx.size()), queue_(64), head_(64, 0)
    {
        const int G = int(idx.size());
        for (int t = 0; t < G; ++t) {
            mask_[t] = gate_mask(g[idx[t]]);
            used_ |= mask_[t];
        }
        for (uint64_t m = used_; m; m &= m - 1) queue_[__builtin_ctzll(m)].reserve(G);
        for (int t = 0; t < G; ++t)
            for (uint64_t m = mask_[t]; m; m &= m - 1) queue_[__builtin_ctzll(m)].push_back(t);
        left_ = G;
    }
    // The next group (gate indices of the caller's list), or false when none is left.
    template <class Fits>
    bool next(Fits fits, std::vector<int> &grp)
    {
        grp.clear();
        if (left_ <= 0) return false;
        uint64_t U = 0;
        for (;;) {
            for (bool again = true; again;) {
                again = false;
                for (uint64_t m = U; m; m &= m - 1) {
                    const int p = __builtin_ctzll(m);
                    for (int t; (t = at_head(p)) >= 0 && !(mask_[t] & ~U) && ready(t);) {
                        grp.push_back(idx_[t]);
                        --left_;
                        for (uint64_t mm = mask_[t]; mm; mm &= mm - 1) ++head_[__builtin_ctzll(mm)];
                        again = true;
                    }
                }
            }
            int best = -1, best_add = 65;
            for (uint64_t pm = used_; pm; pm &= pm - 1) {
                const int t = at_head(__builtin_ctzll(pm));
                if (t < 0 || !ready(t) || !fits(U | mask_[t])) continue;
                const int add = popc(mask_[t] & ~U);
                if (add < best_add || (add == best_add && t < best)) {
                    best_add = add;
                    best = t;
                }
            }
            if (best < 0) break;
            U |= mask_[best];
        }
        return !grp.empty();  // empty only with a gate that `fits` refuses
    }
    // Undo the taking of `gates`, which must be, on each of their qubits, the
    // last ones taken there.
    void give_back(const std::vector<int> &gates)
    {
        if (slot_.empty() && !gates.empty()) {  // formed on first use
            int top = 0;
            for (int gi : idx_) top = std::max(top, gi);
            slot_.assign(size_t(top) + 1, -1);
            for (size_t t = 0; t < idx_.size(); ++t) slot_[size_t(idx_[t])] = int(t);
        }
        for (int gi : gates) {
            const int t = slot_.at(size_t(gi));
            for (uint64_t m = mask_[t]; m; m &= m - 1) --head_[__builtin_ctzll(m)];
            ++left_;
        }
    }

  private:
    int at_head(int p) const { return head_[p] < queue_[p].size() ? queue_[p][head_[p]] : -1; }
    bool ready(int t) const
    {
        for (uint64_t m = mask_[t]; m; m &= m - 1)
            if (at_head(__builtin_ctzll(m)) != t) return false;
        return true;
    }
    const std::vector<int> &idx_;
    std::vector<uint64_t> mask_;
    std::vector<std::vector<int>> queue_;
    std::vector<size_t> head_;
    std::vector<int> slot_;  // caller's gate index -> position in idx (formed by give_back)
    uint64_t used_ = 0;
    int left_ = 0;
};

std::vector<std::vector<int>> frontier_groups(const sv_gate *g, const std::vector<int> &idx, int max_union)
{
    Frontier f(g, idx);
    std::vector<std::vector<int>> out;
    std::vector<int> grp;
    while (f.next([max_union](uint64_t u) { return popc(u) <= max_union; }, grp)) out.push_back(grp);
    return out;
}

// Blocks (positions and members, no matrices) of a list of member groups.
void blocks_of_groups(const sv_gate *g, const std::vector<std::vector<int>> &groups, std::vector<Block> &blocks)
{
    for (const auto &grp : groups) {
        Block B;
        uint64_t m = 0;
        for (int gi : grp) m |= gate_mask(g[gi]);
        for (int p = 0; p < 64; ++p)
            if ((m >> p) & 1) B.q[B.k++] = p;
        B.members = grp;
        blocks.push_back(std::move(B));
    }
}

uint64_t block_mask(const Block &b)
{
    uint64_t m = 0;
    for (int j = 0; j < b.k; ++j) m |= uint64_t(1) << b.q[j];
    return m;
}

// Every block of a tile pass costs a full sweep of the tile in LDS, however
// few qubits it has.  A block is dissolved into a neighbour when the nearest
// earlier block (or, failing that, the nearest later one) that shares a qubit
// with it can take its qubits: the union stays within max_k qubits and the
// neighbour's pass a union that `pass_fits` accepts.  No block in between touches
// its qubits, so its gates commute with everything they move past; they join
// the neighbour's members after (earlier neighbour) or before (later
// neighbour) its own.  Repeated until no block can go.
template <class Fits>
void merge_small_blocks(const sv_gate *g, int max_k, Fits pass_fits, std::vector<Block> &blocks)
{
    (void)g;
    std::vector<uint64_t> mask(blocks.size());
    int n_pass = 0;
    for (size_t i = 0; i < blocks.size(); ++i) {
        mask[i] = block_mask(blocks[i]);
        n_pass = std::max(n_pass, blocks[i].pass + 1);
    }
    std::vector<uint64_t> pass_union(size_t(n_pass), 0);  // positions of each pass's blocks
    auto recompute = [&](int pass) {
        if (pass < 0) return;
        uint64_t u = 0;
        for (size_t j = 0; j < blocks.size(); ++j)
            if (blocks[j].pass == pass) u |= mask[j];
        pass_union[size_t(pass)] = u;
    };
    for (int p = 0; p < n_pass; ++p) recompute(p);
    auto fits = [&](size_t into, uint64_t add) {
        if (popc(mask[into] | add) > max_k) return false;
        const int pass = blocks[into].pass;
        return pass < 0 || pass_fits(pass_union[size_t(pass)] | add);
    };
    for (bool changed = true; changed;) {
        changed = false;
        for (size_t i = 0; i < blocks.size() && !changed; ++i) {
            const uint64_t m = mask[i];
            int before = -1, after = -1;
            for (int j = int(i) - 1; j >= 0; --j)
                if (mask[size_t(j)] & m) {
                    before = j;
                    break;
                }
            for (size_t j = i + 1; j < blocks.size(); ++j)
                if (mask[j] & m) {
                    after = int(j);
                    break;
                }
            int into = -1;
            if (before >= 0 && fits(size_t(before), m)) into = before;
            else if (after >= 0 && fits(size_t(after), m)) into = after;
            if (into < 0) continue;
            Block &t = blocks[size_t(into)];
            const uint64_t tm = mask[size_t(into)] | m;
            if (into < int(i)) {
                t.members.insert(t.members.end(), blocks[i].members.begin(), blocks[i].members.end());
            } else {
                std::vector<int> mem = blocks[i].members;
                mem.insert(mem.end(), t.members.begin(), t.members.end());
                t.members.swap(mem);
            }
            t.k = 0;
            for (uint64_t r = tm; r; r &= r - 1) t.q[t.k++] = __builtin_ctzll(r);
            mask[size_t(into)] = tm;
            const int gone = blocks[i].pass;
            blocks.erase(blocks.begin() + long(i));
            mask.erase(mask.begin() + long(i));
            recompute(gone);
            recompute(t.pass);
            changed = true;
        }
    }
}

}  // namespace

double plan_cost(const std::vector<Block> &blocks, const CostTable &cost)
{
    double s = 0;
    for (auto &b : blocks) s += cost.ms[b.k];
    return s;
}

// Apply a canonical gate matrix (on block-local bits lb[0..kg-1], ascending)
// to every column of the D x D canonical block matrix U (in place).  For each
// group of the 2^kg rows the gate mixes, the new row m is the sum over m' of
// G[m][m'] times row m', accumulated as whole rows (contiguous re/im pairs,
// so the inner loop vectorises) in plain real arithmetic: std::complex
// multiplication carries inf/nan recovery that dominates the cost.
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
    std::vector<double> acc(size_t(2) * Dg * D);
    for (int base = 0; base < D; ++base) {
        if (base & tmask) continue;
        std::fill(acc.begin(), acc.end(), 0.0);
        for (int m = 0; m < Dg; ++m) {
            double *__restrict__ out = acc.data() + size_t(2) * m * D;
            for (int mp = 0; mp < Dg; ++mp) {
                const double gr = G[2 * (size_t(m) * Dg + mp)], gi = G[2 * (size_t(m) * Dg + mp) + 1];
                if (gr == 0.0 && gi == 0.0) continue;
                const double *__restrict__ row = U + size_t(2) * (base | off[mp]) * D;
                for (int c = 0; c < D; ++c) {
                    out[2 * c] += gr * row[2 * c] - gi * row[2 * c + 1];
                    out[2 * c + 1] += gr * row[2 * c + 1] + gi * row[2 * c];
                }
            }
        }
        for (int m = 0; m < Dg; ++m)
            std::copy(acc.begin() + size_t(2) * m * D, acc.begin() + size_t(2) * (m + 1) * D,
                      U + size_t(2) * (base | off[m]) * D);
    }
}

// Embed an m-bit operator V (2^m x 2^m) into m + 1 bits with a new identity
// bit at local position p (bits >= p shift up by one).
static void insert_identity_bit(std::vector<cd> &V, int m, int p)
{
    const int d = 1 << m, d2 = 2 * d;
    std::vector<cd> W(size_t(d2) * d2, cd(0));
    const int lo = (1 << p) - 1;
    auto spread = [&](int x, int bit) { return ((x & ~lo) << 1) | (bit << p) | (x & lo); };
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            const cd v = V[size_t(r) * d + c];
            if (v == cd(0)) continue;
            W[size_t(spread(r, 0)) * d2 + spread(c, 0)] = v;
            W[size_t(spread(r, 1)) * d2 + spread(c, 1)] = v;
        }
    V.swap(W);
}

void block_matrix(const sv_gate *g, Block &b)
{
    // The product is formed on the block bits touched so far (S, ascending):
    // the block matrix is V (on S) times the identity on the untouched bits,
    // so early gates act on a small V.
    std::vector<int> S;               // block-local bits of V, ascending
    std::vector<cd> V(1, cd(1));      // 1 x 1 identity
    std::vector<cd> G;
    for (int gi : b.members) {
        int sq[SV_MAX_K];
        gate_matrix_canonical(g[gi], G, sq);
        int lb[SV_MAX_K];
        for (int j = 0; j < g[gi].k; ++j) {
            int r = 0;
            while (b.q[r] != sq[j]) ++r;
            // grow S by block bit r if the gate touches it first
            auto it = std::lower_bound(S.begin(), S.end(), r);
            if (it == S.end() || *it != r) {
                const int p = int(it - S.begin());
                insert_identity_bit(V, int(S.size()), p);
                S.insert(it, r);
            }
        }
        for (int j = 0; j < g[gi].k; ++j) {
            int r = 0;
            while (b.q[r] != sq[j]) ++r;
            lb[j] = int(std::lower_bound(S.begin(), S.end(), r) - S.begin());
        }
        apply_to_columns(V, int(S.size()), G, g[gi].k, lb);
    }
    // embed V into the full block: entries agree on the untouched bits
    const int D = 1 << b.k, m = int(S.size()), d = 1 << m;
    int smask = 0;
    for (int r : S) smask |= 1 << r;
    int dep[1 << SV_MAX_K];  // V index -> block index
    for (int x = 0; x < d; ++x) {
        int y = 0;
        for (int j = 0; j < m; ++j)
            if ((x >> j) & 1) y |= 1 << S[j];
        dep[x] = y;
    }
    b.m.assign(size_t(D) * D, cd(0));
    for (int rest = 0; rest < D; ++rest) {
        if (rest & smask) continue;
        for (int r = 0; r < d; ++r)
            for (int c = 0; c < d; ++c) b.m[size_t(rest | dep[r]) * D + (rest | dep[c])] = V[size_t(r) * d + c];
    }
}

// Matrices of all blocks; they are independent, so large jobs are spread
// over host threads.
static int block_matrices(const sv_gate *g, std::vector<Block> &blocks)
{
    size_t work = 0;
    for (const auto &B : blocks) work += B.members.size() << (2 * B.k);
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

int fuse_gates(const sv_gate *g, int G, int n, int max_k, int rule, const CostTable &cost,
               std::vector<Block> &blocks, bool with_matrices, int precision)
{
    if (max_k < 1 || max_k > SV_MAX_K) return fail(SV_ERR_ARG, "max_k %d outside 1..%d", max_k, SV_MAX_K);
    if (rule != SV_RULE_PAPER && rule != SV_RULE_ENHANCED && rule != SV_RULE_NONE && rule != SV_RULE_TILED)
        return fail(SV_ERR_ARG, "unknown fusion rule %d", rule);
    if (rule == SV_RULE_TILED) max_k = max_k < 4 ? max_k : 4;  // tile kernels take blocks of <= 4 qubits
    blocks.clear();
    if (rule == SV_RULE_TILED) {
        for (int gi = 0; gi < G; ++gi)
            if (g[gi].k > max_k)
                return fail(SV_ERR_ARG, "gate %d acts on %d qubits, more than max_k=%d", gi, g[gi].k, max_k);
        // Passes one at a time: the next union group, cut into blocks; a pass
        // keeps at most `cap` blocks (what one tile launch holds), and the
        // gates of any further blocks go back to the frontier, so that the
        // next pass can take them with its own gates.  They follow the kept
        // blocks on every qubit they share, so on each of their qubits they
        // are the last gates taken.
        const size_t cap = size_t(std::max(1, tile_pass_capacity(precision)));
        std::vector<int> all(G);
        for (int i = 0; i < G; ++i) all[i] = i;
        Frontier passes(g, all);
        std::vector<int> pg;
        int pass = 0;
        const int tile_bits = tile_pass_bits(), limit = tile_union_limit();
        auto pass_fits = [n, tile_bits, limit](uint64_t u) { return tile_union_fits(u, n, tile_bits, limit); };
        while (passes.next(pass_fits, pg)) {
            const auto sub = frontier_groups(g, pg, max_k);
            const size_t e = std::min(sub.size(), cap);
            const size_t first = blocks.size();
            blocks_of_groups(g, std::vector<std::vector<int>>(sub.begin(), sub.begin() + e), blocks);
            if (e >= 2) {
                for (size_t b = first; b < blocks.size(); ++b) blocks[b].pass = pass;
                ++pass;
            }
            std::vector<int> back;
            for (size_t c = e; c < sub.size(); ++c) back.insert(back.end(), sub[c].begin(), sub[c].end());
            passes.give_back(back);
        }
        merge_small_blocks(g, max_k, pass_fits, blocks);
        return with_matrices ? block_matrices(g, blocks) : SV_OK;
    }
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
    blocks.resize(wb.size());
    for (size_t b = 0; b < wb.size(); ++b) {
        Block &B = blocks[b];
        B.k = 0;
        for (int p = 0; p < 64; ++p)
            if ((wb[b].mask >> p) & 1) B.q[B.k++] = p;
        B.members = wb[b].members;
    }
    if (rule == SV_RULE_ENHANCED) {
        // the frontier plan replaces it when the cost table prices it lower
        std::vector<int> all(G);
        for (int i = 0; i < G; ++i) all[i] = i;
        std::vector<Block> alt;
        blocks_of_groups(g, frontier_groups(g, all, max_k), alt);
        const double ca = plan_cost(alt, cost), cb = plan_cost(blocks, cost);
        if (ca < cb - 1e-12 || (ca <= cb + 1e-12 && alt.size() < blocks.size())) blocks.swap(alt);
    }
    return with_matrices ? block_matrices(g, blocks) : SV_OK;
}


std::vector<std::vector<size_t>> tile_groups(const std::vector<Block> &blocks, int n)
{
    // consecutive blocks of one tile pass; states below 14 qubits (one tile
    // would hold the whole state several times over) apply every block alone
    constexpr int kMinQubits = 14;
    std::vector<std::vector<size_t>> out;
    for (size_t i = 0; i < blocks.size(); ++i) {
        if (n >= kMinQubits && blocks[i].pass >= 0 && !out.empty() && blocks[out.back().back()].pass == blocks[i].pass)
            out.back().push_back(i);
        else
            out.push_back({i});
    }
    return out;
}

double tiled_plan_cost(const std::vector<Block> &blocks, int n, const CostTable &cost)
{
    double c = 0;
    for (const auto &grp : tile_groups(blocks, n)) {
        if (grp.size() > 1) {
            c += cost.tile[grp.size()];
            continue;
        }
        // a block alone runs as a one-block tile pass where that is cheaper
        const int k = blocks[grp[0]].k;
        c += k <= 4 && n >= 14 ? std::min(cost.ms[k], cost.tile[1]) : cost.ms[k];
    }
    return c;
}

}  // namespace sv
