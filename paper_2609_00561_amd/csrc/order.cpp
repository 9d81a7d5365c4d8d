// Host-side ordering for block-multicolored ICCG: ABMC and Leiden blocking,
// greedy block coloring, color-major numbering and the symmetric permutation.
//
// Paper sections: ABMC blocking and block coloring (Section 3, block size
// s = ceil(n/n_b) in Section 6.1); Leiden with modularity, Eq. (1), or the
// constant Potts model, Eq. (2) (Section 4); Leiden settings and the
// descending-size block numbering (Section 7.1).  Leiden itself follows
// Traag, Waltman and van Eck (2019): move nodes fast, refine, aggregate.
//
// The ordering is fully deterministic for a given input and seed; see the
// comments on each routine for the tie-break rules.
#include "iccg_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <numeric>
#include <set>
#include <vector>

namespace iccg {
namespace {

// SplitMix64 (Steele, Lea and Flood 2014).
struct SplitMix64 {
    uint64_t state;
    explicit SplitMix64(uint64_t s) : state(s) {}
    uint64_t next() {
        state += 0x9E3779B97F4A7C15ULL;
        uint64_t z = state;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        return z ^ (z >> 31);
    }
    // Fisher-Yates from the back: position i swaps with next() mod (i+1).
    void shuffle(std::vector<int> &v) {
        for (size_t i = v.size(); i-- > 1;) {
            size_t j = static_cast<size_t>(next() % static_cast<uint64_t>(i + 1));
            std::swap(v[i], v[j]);
        }
    }
    double uniform01() { return static_cast<double>(next() >> 11) * 0x1.0p-53; }
};

// ---------------------------------------------------------------------------
// ABMC
// ---------------------------------------------------------------------------
// Blocks of exactly s nodes (the last may be smaller).  A block is seeded at
// the lowest-numbered unassigned node and grows breadth first: each node that
// joins appends its unassigned, not yet queued neighbours in ascending order.
// An exhausted frontier re-seeds the same block; a full block drops its
// frontier.
std::vector<int> abmc_blocks(int n, const int *rowptr, const int *col, int s) {
    std::vector<int> blk(n, -1);
    std::vector<char> queued(n, 0);
    std::deque<int> frontier;
    std::vector<int> touched;
    int next_seed = 0, nassigned = 0, b = 0;
    if (s < 1) s = 1;
    while (nassigned < n) {
        frontier.clear();
        touched.clear();
        for (int size = 0; size < s && nassigned < n; ++size) {
            int v;
            if (frontier.empty()) {
                while (blk[next_seed] != -1) ++next_seed;
                v = next_seed;
            } else {
                v = frontier.front();
                frontier.pop_front();
            }
            blk[v] = b;
            ++nassigned;
            for (int k = rowptr[v]; k < rowptr[v + 1]; ++k) {
                const int u = col[k];
                if (u != v && blk[u] == -1 && !queued[u]) {
                    queued[u] = 1;
                    frontier.push_back(u);
                    touched.push_back(u);
                }
            }
        }
        for (int u : touched) queued[u] = 0;
        ++b;
    }
    return blk;
}

// ---------------------------------------------------------------------------
// Greedy block coloring: ascending block id, smallest color unused by the
// already-colored adjacent blocks.
// ---------------------------------------------------------------------------
std::vector<int> greedy_block_colors(int n, const int *rowptr, const int *col,
                                     const std::vector<int> &blk, int nb) {
    // block adjacency as sorted unique (b, b') pairs with b' < b
    std::vector<uint64_t> pairs;
    pairs.reserve(static_cast<size_t>(rowptr[n]));
    for (int i = 0; i < n; ++i)
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            const int a = blk[i], c = blk[col[k]];
            if (c < a) pairs.push_back((static_cast<uint64_t>(a) << 32) | static_cast<uint32_t>(c));
        }
    std::sort(pairs.begin(), pairs.end());
    pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());
    std::vector<int> color(nb, -1);
    std::vector<int> used;  // used[c] == b+1 if color c is taken for block b
    size_t p = 0;
    for (int b = 0; b < nb; ++b) {
        for (; p < pairs.size() && static_cast<int>(pairs[p] >> 32) == b; ++p) {
            const int nbc = color[static_cast<int>(pairs[p] & 0xffffffffu)];
            if (nbc >= static_cast<int>(used.size())) used.resize(nbc + 1, 0);
            used[nbc] = b + 1;
        }
        int c = 0;
        while (c < static_cast<int>(used.size()) && used[c] == b + 1) ++c;
        color[b] = c;
    }
    return color;
}

// ---------------------------------------------------------------------------
// Color-major numbering: colors ascending, blocks of a color in ascending id,
// rows of a block in ascending original index.
// ---------------------------------------------------------------------------
void color_major(int n, const std::vector<int> &blk, const std::vector<int> &color,
                 int *perm, int *nblocks, int *block_ptr, int *ncolors, int *color_ptr) {
    const int nb = static_cast<int>(color.size());
    std::vector<int> seq(nb);
    std::iota(seq.begin(), seq.end(), 0);
    std::stable_sort(seq.begin(), seq.end(), [&](int a, int b) { return color[a] < color[b]; });
    const int nc = nb ? *std::max_element(color.begin(), color.end()) + 1 : 0;
    std::vector<int> size(nb, 0);
    for (int i = 0; i < n; ++i) size[blk[i]]++;
    std::vector<int> first(nb);
    int pos = 0, cc = -1;
    for (int q = 0; q < nb; ++q) {
        const int b = seq[q];
        while (cc < color[b]) color_ptr[++cc] = q;
        block_ptr[q] = pos;
        first[b] = pos;
        pos += size[b];
    }
    block_ptr[nb] = pos;
    color_ptr[nc] = nb;
    for (int i = 0; i < n; ++i) perm[first[blk[i]]++] = i;
    *nblocks = nb;
    *ncolors = nc;
}

// ---------------------------------------------------------------------------
// Leiden
// ---------------------------------------------------------------------------
struct WGraph {
    int n = 0;
    std::vector<int64_t> off;   // n+1
    std::vector<int> nbr;       // ascending per node, no self loops
    std::vector<int64_t> wt;
    std::vector<int64_t> nodew;
};

class Leiden {
public:
    Leiden(int quality, double gamma, double beta, double twom, uint64_t seed)
        : md_(quality == ICCG_QUALITY_MODULARITY), gamma_(gamma), beta_(beta), twom_(twom),
          rng_(seed) {}

    // Quality change (up to a positive factor) of joining an isolated node of
    // weight a to a community of weight b with w edges between them:
    // w - gamma*a*b (CPM) or w - gamma*a*b/(2m) (modularity).
    double penalty(int64_t a, int64_t b) const {
        const double t = (gamma_ * static_cast<double>(a)) * static_cast<double>(b);
        return md_ ? t / twom_ : t;
    }

    void move_nodes(const WGraph &g, std::vector<int> &comm);
    void refine(const WGraph &g, const std::vector<int> &comm, std::vector<int> &rc);
    SplitMix64 &rng() { return rng_; }

private:
    bool md_;
    double gamma_, beta_, twom_;
    SplitMix64 rng_;
};

// Move nodes fast: queue = random permutation; each node leaves its community
// D and joins the best of D, its neighbouring communities and an empty one.
// Ties keep D, then prefer the smaller community id; the empty option (gain
// exactly 0) wins only if every other gain is negative and then takes the
// smallest free id.  A moved node re-queues its neighbours outside its new
// community that are not queued.
void Leiden::move_nodes(const WGraph &g, std::vector<int> &comm) {
    const int n = g.n;
    std::vector<int64_t> cw(n, 0);
    std::vector<int> cn(n, 0);
    for (int v = 0; v < n; ++v) { cw[comm[v]] += g.nodew[v]; cn[comm[v]]++; }
    std::set<int> empties;
    for (int c = 0; c < n; ++c) if (cn[c] == 0) empties.insert(c);

    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    rng_.shuffle(order);
    std::deque<int> queue(order.begin(), order.end());
    std::vector<char> queued(n, 1);

    std::vector<int64_t> acc(n, 0);
    std::vector<int> seen(n, -1), nb_comms;
    while (!queue.empty()) {
        const int v = queue.front();
        queue.pop_front();
        queued[v] = 0;
        const int D = comm[v];
        nb_comms.clear();
        for (int64_t e = g.off[v]; e < g.off[v + 1]; ++e) {
            const int c = comm[g.nbr[e]];
            if (seen[c] != v) { seen[c] = v; acc[c] = 0; nb_comms.push_back(c); }
            acc[c] += g.wt[e];
        }
        cw[D] -= g.nodew[v];
        if (--cn[D] == 0) empties.insert(D);
        int best = D;
        double best_gain = static_cast<double>(seen[D] == v ? acc[D] : 0) - penalty(g.nodew[v], cw[D]);
        for (int c : nb_comms) {
            if (c == D) continue;
            const double gain = static_cast<double>(acc[c]) - penalty(g.nodew[v], cw[c]);
            if (gain > best_gain || (gain == best_gain && best != D && c < best)) {
                best = c;
                best_gain = gain;
            }
        }
        if (best_gain < 0.0) best = *empties.begin();
        cw[best] += g.nodew[v];
        if (cn[best]++ == 0) empties.erase(best);
        comm[v] = best;
        if (best != D) {
            for (int64_t e = g.off[v]; e < g.off[v + 1]; ++e) {
                const int u = g.nbr[e];
                if (!queued[u] && comm[u] != best) { queued[u] = 1; queue.push_back(u); }
            }
        }
    }
}

// Refinement inside every community S (ascending id), from singletons: the
// well-connected nodes of S (E(v, S-v) >= penalty(|v|, |S|-|v|)) are visited
// in random order; one that is still alone may merge into a well-connected
// refined community of S next to it (or stay), with probability proportional
// to exp((gain - max gain)/beta) over the options with gain >= 0, drawn by one
// uniform number against the running sum in ascending community id.
void Leiden::refine(const WGraph &g, const std::vector<int> &comm, std::vector<int> &rc) {
    const int n = g.n;
    rc.resize(n);
    std::iota(rc.begin(), rc.end(), 0);
    std::vector<int64_t> rw(g.nodew.begin(), g.nodew.end());
    std::vector<int> rn(n, 1);
    std::vector<int64_t> rcut(n, 0), vcut(n, 0);

    // members per community by counting sort (ascending node id)
    std::vector<int> start(n + 1, 0), members(n);
    for (int v = 0; v < n; ++v) start[comm[v] + 1]++;
    std::partial_sum(start.begin(), start.end(), start.begin());
    {
        std::vector<int> pos(start.begin(), start.end() - 1);
        for (int v = 0; v < n; ++v) members[pos[comm[v]]++] = v;
    }
    std::vector<int64_t> acc(n, 0);
    std::vector<int> seen(n, -1), adj_rc, candidates;
    std::vector<double> gains;
    std::vector<std::pair<int, double>> opts;
    std::vector<int> wellc;
    for (int S = 0; S < n; ++S) {
        const int b0 = start[S], b1 = start[S + 1];
        if (b0 == b1) continue;
        int64_t sw = 0;
        for (int m = b0; m < b1; ++m) sw += g.nodew[members[m]];
        wellc.clear();
        for (int m = b0; m < b1; ++m) {
            const int v = members[m];
            int64_t cut = 0;
            for (int64_t e = g.off[v]; e < g.off[v + 1]; ++e)
                if (comm[g.nbr[e]] == S) cut += g.wt[e];
            vcut[v] = rcut[v] = cut;
            if (static_cast<double>(cut) >= penalty(g.nodew[v], sw - g.nodew[v])) wellc.push_back(v);
        }
        rng_.shuffle(wellc);
        for (int v : wellc) {
            if (rn[rc[v]] != 1) continue;
            adj_rc.clear();
            for (int64_t e = g.off[v]; e < g.off[v + 1]; ++e) {
                const int u = g.nbr[e];
                if (comm[u] != S) continue;
                const int c = rc[u];
                if (seen[c] != v) { seen[c] = v; acc[c] = 0; adj_rc.push_back(c); }
                acc[c] += g.wt[e];
            }
            opts.clear();
            opts.emplace_back(v, 0.0);
            for (int c : adj_rc) {
                if (c == v) continue;
                if (!(static_cast<double>(rcut[c]) >= penalty(rw[c], sw - rw[c]))) continue;
                const double gain = static_cast<double>(acc[c]) - penalty(g.nodew[v], rw[c]);
                if (gain >= 0.0) opts.emplace_back(c, gain);
            }
            std::sort(opts.begin(), opts.end(),
                      [](const std::pair<int, double> &a, const std::pair<int, double> &b) {
                          return a.first < b.first;
                      });
            double gmax = 0.0;
            for (const auto &o : opts) gmax = std::max(gmax, o.second);
            double total = 0.0;
            for (const auto &o : opts) total += std::exp((o.second - gmax) / beta_);
            const double threshold = rng_.uniform01() * total;
            int target = opts.back().first;
            double run = 0.0;
            for (const auto &o : opts) {
                run += std::exp((o.second - gmax) / beta_);
                if (run >= threshold) { target = o.first; break; }
            }
            if (target != v) {
                const int64_t w_vt = (seen[target] == v) ? acc[target] : 0;
                rn[v] = 0;
                rw[v] = 0;
                rc[v] = target;
                rn[target] += 1;
                rw[target] += g.nodew[v];
                rcut[target] += vcut[v] - 2 * w_vt;
            }
        }
    }
}

// Relabel to 0..k-1 by first appearance over ascending node id (ascending
// smallest member); ids lie in [0, id_bound).
int relabel_by_first_member(std::vector<int> &labels, int id_bound) {
    std::vector<int> fresh(id_bound, -1);
    int k = 0;
    for (int &x : labels) {
        if (fresh[x] < 0) fresh[x] = k++;
        x = fresh[x];
    }
    return k;
}

// One node per refined community (already relabelled 0..k-1); integer sums
// of node and edge weights; edges inside a refined community are dropped.
WGraph aggregate(const WGraph &g, const std::vector<int> &rc, int k) {
    WGraph h;
    h.n = k;
    h.nodew.assign(k, 0);
    std::vector<int> start(k + 1, 0), members(g.n);
    for (int v = 0; v < g.n; ++v) { h.nodew[rc[v]] += g.nodew[v]; start[rc[v] + 1]++; }
    std::partial_sum(start.begin(), start.end(), start.begin());
    {
        std::vector<int> pos(start.begin(), start.end() - 1);
        for (int v = 0; v < g.n; ++v) members[pos[rc[v]]++] = v;
    }
    h.off.assign(k + 1, 0);
    std::vector<int64_t> acc(k, 0);
    std::vector<int> seen(k, -1), list;
    for (int a = 0; a < k; ++a) {
        list.clear();
        for (int m = start[a]; m < start[a + 1]; ++m) {
            const int v = members[m];
            for (int64_t e = g.off[v]; e < g.off[v + 1]; ++e) {
                const int b = rc[g.nbr[e]];
                if (b == a) continue;
                if (seen[b] != a) { seen[b] = a; acc[b] = 0; list.push_back(b); }
                acc[b] += g.wt[e];
            }
        }
        std::sort(list.begin(), list.end());
        for (int b : list) { h.nbr.push_back(b); h.wt.push_back(acc[b]); }
        h.off[a + 1] = static_cast<int64_t>(h.nbr.size());
    }
    return h;
}

std::vector<int> leiden(int n, const int *rowptr, const int *col, int quality, double gamma,
                        double beta, int n_iter, uint64_t seed) {
    WGraph g0;
    g0.n = n;
    g0.off.assign(n + 1, 0);
    g0.nodew.assign(n, 0);
    for (int i = 0; i < n; ++i) {
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
            if (col[k] != i) { g0.nbr.push_back(col[k]); g0.wt.push_back(1); }
        g0.off[i + 1] = static_cast<int64_t>(g0.nbr.size());
        g0.nodew[i] = (quality == ICCG_QUALITY_MODULARITY) ? (g0.off[i + 1] - g0.off[i]) : 1;
    }
    Leiden L(quality, gamma, beta, static_cast<double>(g0.off[n]), seed);

    std::vector<int> part(n);
    std::iota(part.begin(), part.end(), 0);
    for (int it = 0; it < n_iter; ++it) {
        WGraph level;
        const WGraph *G = &g0;
        std::vector<int> comm = part;          // partition of G's nodes
        std::vector<int> where(n);             // original node -> node of G
        std::iota(where.begin(), where.end(), 0);
        for (;;) {
            L.move_nodes(*G, comm);
            std::vector<char> present(G->n, 0);
            int ncomm = 0;
            for (int c : comm) if (!present[c]) { present[c] = 1; ++ncomm; }
            if (ncomm == G->n) break;
            std::vector<int> rc;
            L.refine(*G, comm, rc);
            const int k = relabel_by_first_member(rc, G->n);
            if (k == G->n) break;
            WGraph next = aggregate(*G, rc, k);
            std::vector<int> next_comm(k);
            for (int v = 0; v < G->n; ++v) next_comm[rc[v]] = comm[v];
            relabel_by_first_member(next_comm, G->n);
            for (int &w : where) w = rc[w];
            level = std::move(next);
            G = &level;
            comm.swap(next_comm);
        }
        const int bound = G->n;
        for (int i = 0; i < n; ++i) part[i] = comm[where[i]];
        relabel_by_first_member(part, bound);
    }
    return part;
}

// Section 7.1: larger blocks get smaller numbers; equal sizes keep the order
// of their smallest original node.
void renumber_by_size(std::vector<int> &blk, int nb) {
    std::vector<int> size(nb, 0), minv(nb, -1);
    for (int i = 0; i < static_cast<int>(blk.size()); ++i) {
        size[blk[i]]++;
        if (minv[blk[i]] < 0) minv[blk[i]] = i;
    }
    std::vector<int> ids(nb);
    std::iota(ids.begin(), ids.end(), 0);
    std::sort(ids.begin(), ids.end(), [&](int a, int b) {
        return size[a] != size[b] ? size[a] > size[b] : minv[a] < minv[b];
    });
    std::vector<int> rank(nb);
    for (int r = 0; r < nb; ++r) rank[ids[r]] = r;
    for (int &b : blk) b = rank[b];
}

int check_pattern_args(int n, const int *rowptr, const int *col) {
    if (n < 0 || (n > 0 && (!rowptr || !col))) return set_error(ICCG_EINVAL, "null pattern");
    if (n == 0) return ICCG_OK;
    if (rowptr[0] != 0) return set_error(ICCG_EINVAL, "rowptr[0] must be 0");
    for (int i = 0; i < n; ++i) {
        if (rowptr[i + 1] < rowptr[i]) return set_error(ICCG_EINVAL, "rowptr not monotone");
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
            if (col[k] < 0 || col[k] >= n) return set_error(ICCG_EINVAL, "column index out of range");
    }
    return ICCG_OK;
}

}  // namespace
}  // namespace iccg

using namespace iccg;

extern "C" int iccg_order_abmc(int n, const int *rowptr, const int *col, int block_size,
                               int *perm, int *nblocks, int *block_ptr, int *ncolors,
                               int *color_ptr) {
    try {
        if (int st = check_pattern_args(n, rowptr, col)) return st;
        if (block_size < 1) return set_error(ICCG_EINVAL, "block_size must be >= 1");
        if (!perm || !nblocks || !block_ptr || !ncolors || !color_ptr)
            return set_error(ICCG_EINVAL, "null output");
        if (n == 0) { *nblocks = 0; *ncolors = 0; block_ptr[0] = 0; color_ptr[0] = 0; return ICCG_OK; }
        std::vector<int> blk = abmc_blocks(n, rowptr, col, block_size);
        const int nb = *std::max_element(blk.begin(), blk.end()) + 1;
        std::vector<int> color = greedy_block_colors(n, rowptr, col, blk, nb);
        color_major(n, blk, color, perm, nblocks, block_ptr, ncolors, color_ptr);
        return ICCG_OK;
    } catch (const std::bad_alloc &) {
        return set_error(ICCG_ENOMEM, "host allocation failed in iccg_order_abmc");
    }
}

extern "C" int iccg_order_leiden(int n, const int *rowptr, const int *col, int quality,
                                 double gamma, double beta, int n_iter, uint64_t seed, int *perm,
                                 int *nblocks, int *block_ptr, int *ncolors, int *color_ptr) {
    try {
        if (int st = check_pattern_args(n, rowptr, col)) return st;
        if (quality != ICCG_QUALITY_MODULARITY && quality != ICCG_QUALITY_CPM)
            return set_error(ICCG_EINVAL, "quality must be modularity (0) or CPM (1)");
        if (!(gamma >= 0.0) || !(beta > 0.0) || n_iter < 1)
            return set_error(ICCG_EINVAL, "need gamma >= 0, beta > 0, n_iter >= 1");
        if (!perm || !nblocks || !block_ptr || !ncolors || !color_ptr)
            return set_error(ICCG_EINVAL, "null output");
        if (n == 0) { *nblocks = 0; *ncolors = 0; block_ptr[0] = 0; color_ptr[0] = 0; return ICCG_OK; }
        std::vector<int> blk = leiden(n, rowptr, col, quality, gamma, beta, n_iter, seed);
        const int nb = *std::max_element(blk.begin(), blk.end()) + 1;
        renumber_by_size(blk, nb);
        std::vector<int> color = greedy_block_colors(n, rowptr, col, blk, nb);
        color_major(n, blk, color, perm, nblocks, block_ptr, ncolors, color_ptr);
        return ICCG_OK;
    } catch (const std::bad_alloc &) {
        return set_error(ICCG_ENOMEM, "host allocation failed in iccg_order_leiden");
    }
}

extern "C" int iccg_permute(int n, const int *rowptr, const int *col, const double *val,
                            const int *perm, int *prow, int *pcol, double *pval) {
    try {
        if (int st = check_pattern_args(n, rowptr, col)) return st;
        if (!val || !perm || !prow || !pcol || !pval) return set_error(ICCG_EINVAL, "null argument");
        std::vector<int> inv(n, -1);
        for (int i = 0; i < n; ++i) {
            if (perm[i] < 0 || perm[i] >= n || inv[perm[i]] != -1)
                return set_error(ICCG_EINVAL, "perm is not a permutation");
            inv[perm[i]] = i;
        }
        std::vector<std::pair<int, double>> row;
        prow[0] = 0;
        for (int i = 0; i < n; ++i) {
            const int o = perm[i];
            row.clear();
            for (int k = rowptr[o]; k < rowptr[o + 1]; ++k) row.emplace_back(inv[col[k]], val[k]);
            std::sort(row.begin(), row.end(),
                      [](const std::pair<int, double> &a, const std::pair<int, double> &b) {
                          return a.first < b.first;
                      });
            int p = prow[i];
            for (const auto &e : row) { pcol[p] = e.first; pval[p] = e.second; ++p; }
            prow[i + 1] = p;
        }
        return ICCG_OK;
    } catch (const std::bad_alloc &) {
        return set_error(ICCG_ENOMEM, "host allocation failed in iccg_permute");
    }
}

// Load-imbalance statistics of an ordering (Section 7.3, Table 6).  The Gini
// sum over ordered pairs, sum_i sum_j |s_i - s_j|, is taken exactly in
// integers from the sorted sizes: the k-th smallest size (0-based) is the
// larger element of k pairs and the smaller of n_b - 1 - k, so the sum is
// 2 sum_k (2k - n_b + 1) s_(k).
extern "C" int iccg_block_stats(int nblocks, const int *block_ptr, int ncolors, const int *color_ptr,
                                double *out) {
    try {
        if (!out || !block_ptr || !color_ptr || nblocks < 1 || ncolors < 1)
            return set_error(ICCG_EINVAL, "need nblocks, ncolors >= 1, block_ptr, color_ptr and out");
        if (block_ptr[0] != 0 || color_ptr[0] != 0 || color_ptr[ncolors] != nblocks)
            return set_error(ICCG_EBADORDER, "block_ptr/color_ptr must start at 0 and color_ptr end at nblocks");
        std::vector<long long> s(nblocks);
        for (int b = 0; b < nblocks; ++b) {
            s[b] = static_cast<long long>(block_ptr[b + 1]) - block_ptr[b];
            if (s[b] <= 0) return set_error(ICCG_EBADORDER, "empty or reversed block");
        }
        const long long n = block_ptr[nblocks];
        long long cmax = 0;
        for (int c = 0; c < ncolors; ++c) {
            if (color_ptr[c + 1] <= color_ptr[c]) return set_error(ICCG_EBADORDER, "empty or reversed color");
            cmax = std::max(cmax, static_cast<long long>(block_ptr[color_ptr[c + 1]]) - block_ptr[color_ptr[c]]);
        }
        std::vector<long long> sorted(s);
        std::sort(sorted.begin(), sorted.end());
        long long pairs = 0;
        for (int k = 0; k < nblocks; ++k) pairs += (2LL * k - nblocks + 1) * sorted[k];
        pairs *= 2;
        const double nb = static_cast<double>(nblocks);
        const double mean_block = static_cast<double>(n) / nb;
        out[0] = nb;
        out[1] = static_cast<double>(ncolors);
        out[2] = static_cast<double>(pairs) / (2.0 * nb * nb * mean_block);
        out[3] = static_cast<double>(sorted.back());
        out[4] = static_cast<double>(sorted.back()) / mean_block;
        out[5] = static_cast<double>(cmax) / (static_cast<double>(n) / static_cast<double>(ncolors));
        return ICCG_OK;
    } catch (const std::bad_alloc &) {
        return set_error(ICCG_ENOMEM, "host allocation failed in iccg_block_stats");
    }
}
