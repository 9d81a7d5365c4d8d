// Host-side setup of the substitution schedules and the host IC(0) factor.
//
// Algorithm 1 (Section 3) runs the colors in sequence, the blocks of one color
// in parallel and the rows of a block in ascending order; the backward sweep
// runs the same scheme in reverse.  Here the blocks of one color are packed
// into wavefront-sized chunks and, inside a chunk, every row gets the level of
// its longest chain of in-chunk dependencies.  Rows of one level only read
// values that are final (earlier colors, earlier chunks, lower levels), so
// computing them together gives each row exactly the terms of the in-order
// sweep.
#include "iccg_internal.h"

#include <algorithm>
#include <cmath>

namespace iccg {

namespace {

struct RowEntries {
    std::vector<int> ext, inn;   // CSR positions: before-chunk / in-chunk dependencies
};

}  // namespace

int build_sweep_plan(bool forward, int n, const int *rowptr, const int *col, const int *tpos,
                     int nblocks, const int *block_ptr, int ncolors, const int *color_ptr,
                     int pack_rows, SweepPlan &out) {
    (void)nblocks;
    out = SweepPlan();
    out.forward = forward;
    out.meta.assign(n, 0);
    if (pack_rows < 1 || pack_rows > kChunkRows) pack_rows = kChunkRows;

    // 1. chunk boundaries, grouped into tasks, color by color
    std::vector<std::pair<int, int>> chunk_rows;   // [row0, row1)
    out.color_task_ptr.push_back(0);
    out.task_chunk_ptr.push_back(0);
    auto close_task = [&]() { out.task_chunk_ptr.push_back(static_cast<int>(chunk_rows.size())); };
    for (int c = 0; c < ncolors; ++c) {
        int open0 = -1, open1 = -1;
        auto flush = [&]() {
            if (open0 >= 0) {
                chunk_rows.emplace_back(open0, open1);
                close_task();
                open0 = open1 = -1;
            }
        };
        for (int b = color_ptr[c]; b < color_ptr[c + 1]; ++b) {
            const int r0 = block_ptr[b], r1 = block_ptr[b + 1], size = r1 - r0;
            if (size > kChunkRows) {
                flush();
                for (int r = r0; r < r1; r += kChunkRows) chunk_rows.emplace_back(r, std::min(r + kChunkRows, r1));
                close_task();
            } else {
                if (open0 >= 0 && (open1 - open0) + size > pack_rows) flush();
                if (open0 < 0) open0 = open1 = r0;
                open1 = r1;
            }
        }
        flush();
        out.color_task_ptr.push_back(static_cast<int>(out.task_chunk_ptr.size()) - 1);
    }

    // 2. per chunk: classify entries, levels, slot layout
    long long nslots = 0;
    RowEntries rows[kChunkRows];
    int level[kChunkRows], wid[kChunkRows], sorted[kChunkRows], pos[kChunkRows];
    for (const auto &cr : chunk_rows) {
        const int r0 = cr.first, r1 = cr.second, nr = r1 - r0;
        int width = 0, depth = 0;
        for (int step = 0; step < nr; ++step) {
            const int t = forward ? step : nr - 1 - step;
            const int i = r0 + t;
            RowEntries &re = rows[t];
            re.ext.clear();
            re.inn.clear();
            int lev = 0;
            for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                const int j = col[k];
                if (forward ? (j >= i) : (j <= i)) continue;
                const bool inside = (j >= r0 && j < r1);
                if (inside) {
                    re.inn.push_back(k);
                    lev = std::max(lev, level[j - r0] + 1);
                } else {
                    re.ext.push_back(k);
                }
            }
            level[t] = lev;
            if (re.ext.size() > kMetaNextMask)
                return set_error(ICCG_EINVAL, "a row has more than 8191 off-diagonal entries in one triangle");
            wid[t] = static_cast<int>(re.ext.size() + re.inn.size());
            width = std::max(width, wid[t]);
            depth = std::max(depth, lev + 1);
        }
        if (width > 0x7fff) return set_error(ICCG_EINVAL, "a row has more than 32767 entries in one triangle");
        Chunk ch{};
        ch.row0 = r0;
        ch.off = static_cast<int32_t>(nslots);
        ch.shape = nr | (width << 16);
        ch.depth = depth;
        // sorted positions and the rows of each slot (see Chunk)
        for (int t = 0; t < nr; ++t) sorted[t] = t;
        if (ch.jagged())
            std::stable_sort(sorted, sorted + nr, [&](int a, int b) { return wid[a] > wid[b]; });
        for (int l = 0; l < nr; ++l) pos[sorted[l]] = l;
        std::vector<long long> first(width + 1, 0);
        for (int k = 0; k < width; ++k) {
            int cnt = nr;
            if (ch.jagged()) {
                cnt = 0;
                for (int t = 0; t < nr; ++t) cnt += wid[t] > k;
                ch.cnt[k >> 2] |= static_cast<uint32_t>(cnt) << (8 * (k & 3));
            }
            first[k + 1] = first[k] + cnt;
        }
        if (nslots + first[width] >= (1LL << 31))
            return set_error(ICCG_EINVAL, "substitution schedule exceeds 2^31 slots");
        out.chunks.push_back(ch);
        out.max_depth = std::max(out.max_depth, depth);
        out.max_width = std::max(out.max_width, width);
        out.slot_col.resize(nslots + first[width], -1);
        out.slot_src.resize(nslots + first[width], -1);
        for (int t = 0; t < nr; ++t) {
            out.meta[r0 + t] = pack_meta(static_cast<int>(rows[t].ext.size()),
                                         static_cast<int>(rows[t].inn.size()), level[t], pos[t]);
            int k = 0;
            for (const auto *grp : {&rows[t].ext, &rows[t].inn})
                for (int q : *grp) {
                    const long long slot = nslots + first[k] + pos[t];
                    out.slot_col[slot] = col[q];
                    out.slot_src[slot] = forward ? q : tpos[q];
                    ++k;
                }
        }
        nslots += first[width];
    }
    const int ntasks = static_cast<int>(out.task_chunk_ptr.size()) - 1;
    // dependency lists: the tasks owning the before-chunk terms of a task's rows
    std::vector<int> task_of_row(n, -1);
    for (int t = 0; t < ntasks; ++t)
        for (int ch = out.task_chunk_ptr[t]; ch < out.task_chunk_ptr[t + 1]; ++ch)
            for (int r = chunk_rows[ch].first; r < chunk_rows[ch].second; ++r) task_of_row[r] = t;
    out.dep_ptr.assign(1, 0);
    std::vector<int> list;
    for (int t = 0; t < ntasks; ++t) {
        list.clear();
        for (int ch = out.task_chunk_ptr[t]; ch < out.task_chunk_ptr[t + 1]; ++ch)
            for (int i = chunk_rows[ch].first; i < chunk_rows[ch].second; ++i)
                for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                    const int j = col[k];
                    if (forward ? (j >= i) : (j <= i)) continue;
                    const int tj = task_of_row[j];
                    if (tj != t) list.push_back(tj);
                }
        std::sort(list.begin(), list.end());
        list.erase(std::unique(list.begin(), list.end()), list.end());
        for (int d : list)
            if (forward ? (d > t) : (d < t))
                return set_error(ICCG_EBADORDER, "a sweep dependency points forward in processing order");
        out.deps.insert(out.deps.end(), list.begin(), list.end());
        out.dep_ptr.push_back(static_cast<int>(out.deps.size()));
    }
    // launch table
    out.wg_task.assign(ntasks, -1);
    int B = 0;
    for (int step = 0; step < ncolors; ++step) {
        const int c = forward ? step : ncolors - 1 - step;
        const int t0 = out.color_task_ptr[c], t1 = out.color_task_ptr[c + 1], T = t1 - t0;
        int cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int b = B; b < B + T; ++b) cnt[b & 7]++;
        int next[8];
        int start = t0;
        for (int x = 0; x < 8; ++x) {
            next[x] = start;
            start += cnt[x];
        }
        for (int b = B; b < B + T; ++b) out.wg_task[b] = next[b & 7]++;
        B += T;
    }
    // Regions of the single-launch sweep (the XCD slot each task is dealt to).
    // Values pass between tasks of one region through that XCD's L2.  A task
    // with a dependency in another region reads all of its before-chunk values
    // with device-coherent loads, so every row such a task reads (its own
    // earlier chunks included) is written through to memory: the export bit.
    std::vector<int> region(ntasks, 0);
    for (int b = 0; b < ntasks; ++b) region[out.wg_task[b]] = b & 7;
    std::vector<int> kind(ntasks, 0);
    for (int t = 0; t < ntasks; ++t)
        for (int d = out.dep_ptr[t]; d < out.dep_ptr[t + 1]; ++d)
            if (region[out.deps[d]] != region[t]) kind[t] |= kTaskRemote;
    for (int t = 0; t < ntasks; ++t) {
        if (!(kind[t] & kTaskRemote)) continue;
        ++out.remote_tasks;
        for (int ch = out.task_chunk_ptr[t]; ch < out.task_chunk_ptr[t + 1]; ++ch) {
            const int r0 = chunk_rows[ch].first, r1 = chunk_rows[ch].second;
            for (int i = r0; i < r1; ++i)
                for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                    const int j = col[k];
                    if (forward ? (j >= i) : (j <= i)) continue;
                    if (j >= r0 && j < r1) continue;
                    if (!(out.meta[j] & kMetaExport)) {
                        out.meta[j] |= kMetaExport;
                        ++out.exported_rows;
                        kind[task_of_row[j]] |= kTaskExports;
                    }
                }
        }
    }
    out.tasks.resize(ntasks);
    for (int t = 0; t < ntasks; ++t) {
        TaskRec &tr = out.tasks[t];
        tr.c0 = out.task_chunk_ptr[t];
        tr.c1 = out.task_chunk_ptr[t + 1];
        const int nd = out.dep_ptr[t + 1] - out.dep_ptr[t];
        if (nd >= (1 << 29)) return set_error(ICCG_EINVAL, "a task has too many dependencies");
        tr.dep0 = out.dep_ptr[t];
        tr.kind_ndeps = kind[t] | (nd << 2);
        tr.wide = -1;
        tr.first = out.chunks[forward ? tr.c0 : tr.c1 - 1];
    }
    return ICCG_OK;
}

int build_wide_plan(SweepPlan &plan, int n, const int *rowptr, const int *col, const int *tpos,
                    int ncolors, int piece_rows, WidePlan &out) {
    out = WidePlan();
    const bool fwd = plan.forward;
    out.color_ptr.assign(1, 0);
    out.piece_ptr.assign(1, 0);
    out.wmeta.assign(n, 0);
    out.wlev.assign(n, 0);
    if (piece_rows < kChunkRows || piece_rows > kWideMaxRows || piece_rows % kChunkRows)
        return set_error(ICCG_EINVAL, "wide piece size");
    std::vector<int> lev(piece_rows);
    std::vector<std::vector<int>> outside(piece_rows), inside(piece_rows);
    for (int c = 0; c < ncolors; ++c) {
        for (int t = plan.color_task_ptr[c]; t < plan.color_task_ptr[c + 1]; ++t) {
            TaskRec &tr = plan.tasks[t];
            if (tr.c1 - tr.c0 < 2) continue;
            // one block [r0, r1) cut into 64-row chunks
            const int r0 = plan.chunks[tr.c0].row0;
            const int r1 = plan.chunks[tr.c1 - 1].row0 + plan.chunks[tr.c1 - 1].nrows();
            if (r1 - r0 <= kWideMinRows) continue;
            tr.wide = static_cast<int>(out.task.size());
            out.task.push_back(t);
            const int npieces = (r1 - r0 + piece_rows - 1) / piece_rows;
            for (int q = 0; q < npieces; ++q) {
                const int pi = fwd ? q : npieces - 1 - q;
                const int p0 = r0 + pi * piece_rows, p1 = std::min(r1, p0 + piece_rows), np = p1 - p0;
                // levels in the sweep's row order
                int depth = 0;
                for (int step = 0; step < np; ++step) {
                    const int u = fwd ? step : np - 1 - step;
                    const int i = p0 + u;
                    outside[u].clear();
                    inside[u].clear();
                    int l = 0;
                    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                        const int j = col[k];
                        if (fwd ? (j >= i) : (j <= i)) continue;
                        if (j >= p0 && j < p1) {
                            inside[u].push_back(k);
                            l = std::max(l, lev[j - p0] + 1);
                        } else {
                            outside[u].push_back(k);
                        }
                    }
                    if (outside[u].size() > 0xffff || inside[u].size() > 0xffff)
                        return set_error(ICCG_EINVAL, "a row has more than 65535 entries in one triangle");
                    lev[u] = l;
                    depth = std::max(depth, l + 1);
                    out.wmeta[i] = static_cast<uint32_t>(outside[u].size()) |
                                   (static_cast<uint32_t>(inside[u].size()) << 16);
                    out.wlev[i] = l;
                }
                WidePiece P{};
                P.sub0 = static_cast<int>(out.subs.size());
                P.depth = depth;
                P.row0 = p0;
                for (int s0 = p0; s0 < p1; s0 += kChunkRows) {
                    const int nr = std::min(kChunkRows, p1 - s0);
                    int width = 0;
                    for (int u = s0 - p0; u < s0 - p0 + nr; ++u)
                        width = std::max(width, static_cast<int>(outside[u].size() + inside[u].size()));
                    const long long off = static_cast<long long>(out.slot_col.size());
                    if (off + static_cast<long long>(width) * nr >= (1LL << 31))
                        return set_error(ICCG_EINVAL, "wide schedule exceeds 2^31 slots");
                    Chunk ch{};
                    ch.row0 = s0;
                    ch.off = static_cast<int32_t>(off);
                    ch.shape = nr | (width << 16);
                    ch.depth = depth;
                    out.subs.push_back(ch);
                    out.slot_col.resize(off + static_cast<long long>(width) * nr, -1);
                    out.slot_src.resize(off + static_cast<long long>(width) * nr, -1);
                    for (int r = 0; r < nr; ++r) {
                        const int u = s0 - p0 + r;
                        int k = 0;
                        for (const auto *grp : {&outside[u], &inside[u]})
                            for (int e : *grp) {
                                const long long slot = off + static_cast<long long>(k) * nr + r;
                                out.slot_col[slot] = col[e];
                                out.slot_src[slot] = fwd ? e : tpos[e];
                                ++k;
                            }
                    }
                }
                P.nsub = static_cast<int>(out.subs.size()) - P.sub0;
                out.pieces.push_back(P);
                out.max_depth = std::max(out.max_depth, depth);
            }
            out.piece_ptr.push_back(static_cast<int>(out.pieces.size()));
        }
        out.color_ptr.push_back(static_cast<int>(out.task.size()));
    }
    return ICCG_OK;
}

// Invariants of a finished sweep plan, re-derived independently of how it was
// built; used by iccg_schedule_stats.  Returns ICCG_OK or an error naming the
// first violation.
int check_sweep_plan(const SweepPlan &P, int n, const int *rowptr, const int *col, int ncolors,
                     const int *block_ptr, const int *color_ptr) {
    const bool fwd = P.forward;
    const int ntasks = static_cast<int>(P.task_chunk_ptr.size()) - 1;
    auto fail = [](const std::string &m) { return set_error(ICCG_EINVAL, "schedule invariant: " + m); };
    if (static_cast<int>(P.tasks.size()) != ntasks || static_cast<int>(P.wg_task.size()) != ntasks)
        return fail("task tables disagree in size");
    // chunks tile each color's rows in order; every row in exactly one chunk
    std::vector<int> task_of_row(n, -1), color_of_task(ntasks, -1);
    for (int c = 0; c < ncolors; ++c) {
        int next = block_ptr[color_ptr[c]];
        for (int t = P.color_task_ptr[c]; t < P.color_task_ptr[c + 1]; ++t) {
            color_of_task[t] = c;
            for (int ch = P.task_chunk_ptr[t]; ch < P.task_chunk_ptr[t + 1]; ++ch) {
                const Chunk &k = P.chunks[ch];
                if (k.row0 != next) return fail("chunks do not tile color " + std::to_string(c));
                const int nr = k.nrows();
                if (nr < 1 || nr > kChunkRows) return fail("chunk row count out of range");
                for (int i = k.row0; i < k.row0 + nr; ++i) task_of_row[i] = t;
                next += nr;
            }
        }
        if (next != block_ptr[color_ptr[c + 1]]) return fail("chunks do not cover color " + std::to_string(c));
    }
    // slots: chunks contiguous; sorted positions a permutation ordered by
    // decreasing entry count (identity for padded chunks); every row's
    // triangle entries, before-chunk ones first, each group ascending; the
    // schedule word's counts agree
    long long next_slot = 0;
    for (size_t ch = 0; ch < P.chunks.size(); ++ch) {
        const Chunk &k = P.chunks[ch];
        const int nr = k.nrows(), W = k.width();
        if (k.off != next_slot) return fail("chunk slots are not contiguous");
        if (!k.jagged() && (k.cnt[0] | k.cnt[1])) return fail("padded chunk with slot counts");
        std::vector<int> cnt(nr), at(nr, -1);
        std::vector<long long> first(W + 1, 0);
        for (int s = 0; s < W; ++s) first[s + 1] = first[s] + k.slot_rows(s);
        for (int t = 0; t < nr; ++t) {
            const int i = k.row0 + t;
            const uint32_t m = P.meta[i];
            const int ne = meta_next(m), ni = meta_inner(m), l = meta_pos(m);
            if (l >= nr || at[l] >= 0) return fail("sorted positions are not a permutation");
            at[l] = t;
            if (!k.jagged() && l != t) return fail("padded chunk with moved rows");
            for (int q = rowptr[i]; q < rowptr[i + 1]; ++q)
                if (fwd ? col[q] < i : col[q] > i) ++cnt[t];
            if (ne + ni != cnt[t] || cnt[t] > W) return fail("row " + std::to_string(i) + " entry counts");
            int prev = -1;
            for (int s = 0; s < W; ++s) {
                if ((l < k.slot_rows(s)) != (s < cnt[t] || !k.jagged()))
                    return fail("slot counts disagree with row " + std::to_string(i));
                if (l >= k.slot_rows(s)) continue;
                const int c = P.slot_col[k.off + first[s] + l];
                if (s >= cnt[t]) {
                    if (c != -1) return fail("padding slot holds an entry");
                    continue;
                }
                const bool inside = c >= k.row0 && c < k.row0 + nr;
                if (inside != (s >= ne)) return fail("slot group order in row " + std::to_string(i));
                if (s == ne) prev = -1;
                if (c <= prev) return fail("slots not ascending in row " + std::to_string(i));
                prev = c;
            }
        }
        for (int l = 1; l < nr; ++l)
            if (k.jagged() && cnt[at[l]] > cnt[at[l - 1]]) return fail("sorted positions out of order");
        next_slot += first[W];
    }
    if (next_slot != static_cast<long long>(P.slot_col.size())) return fail("slot array size");
    // launch table: a permutation, colors in processing order; every
    // dependency an earlier color and an earlier position
    std::vector<int> pos(ntasks, -1);
    for (int b = 0; b < ntasks; ++b) {
        const int t = P.wg_task[b];
        if (t < 0 || t >= ntasks || pos[t] >= 0) return fail("launch table is not a permutation");
        pos[t] = b;
    }
    for (int t = 0; t < ntasks; ++t) {
        const int d0 = P.tasks[t].dep0, nd = P.tasks[t].kind_ndeps >> 2;
        if (d0 != P.dep_ptr[t] || d0 + nd != P.dep_ptr[t + 1]) return fail("task dependency range");
        for (int d = d0; d < d0 + nd; ++d) {
            const int u = P.deps[d];
            if (pos[u] >= pos[t]) return fail("a dependency is not at an earlier position");
            const bool earlier = fwd ? color_of_task[u] < color_of_task[t] : color_of_task[u] > color_of_task[t];
            if (!earlier && u != t) return fail("a dependency is not in an earlier color");
        }
    }
    // every row a task reads across chunks comes from its dependencies or its
    // own earlier chunks; rows read by remote tasks are exported
    for (int t = 0; t < ntasks; ++t) {
        const bool remote = P.tasks[t].kind_ndeps & kTaskRemote;
        const int d0 = P.tasks[t].dep0, nd = P.tasks[t].kind_ndeps >> 2;
        for (int ch = P.task_chunk_ptr[t]; ch < P.task_chunk_ptr[t + 1]; ++ch) {
            const Chunk &k = P.chunks[ch];
            const int nr = k.shape & 0xffff;
            for (int i = k.row0; i < k.row0 + nr; ++i)
                for (int q = rowptr[i]; q < rowptr[i + 1]; ++q) {
                    const int j = col[q];
                    if (fwd ? j >= i : j <= i) continue;
                    if (j >= k.row0 && j < k.row0 + nr) continue;
                    const int u = task_of_row[j];
                    if (u != t && !std::binary_search(P.deps.begin() + d0, P.deps.begin() + d0 + nd, u))
                        return fail("row " + std::to_string(i) + " reads a task it does not wait for");
                    if (remote && !(P.meta[j] & kMetaExport)) return fail("a row read remotely is not exported");
                    if (remote && !(P.tasks[u].kind_ndeps & kTaskExports))
                        return fail("a task with exported rows lacks the export kind");
                }
        }
    }
    return ICCG_OK;
}

// Launch order of the slices: the k-th eighth of every color's rows goes to
// the k-th eighth of the launch, so the workgroups that one XCD runs cover the
// same region of the domain in every color, and the values they gather from
// the other colors share that XCD's L2.
static std::vector<int> slice_launch_order(int n, int ns, const int *block_ptr, int ncolors,
                                           const int *color_ptr) {
    std::vector<int> c_row0(ncolors), c_rows(ncolors);
    for (int c = 0; c < ncolors; ++c) {
        c_row0[c] = block_ptr[color_ptr[c]];
        c_rows[c] = block_ptr[color_ptr[c + 1]] - c_row0[c];
    }
    std::vector<long long> key(ns);
    int c = 0;
    for (int s = 0; s < ns; ++s) {
        const int r = std::min(n - 1, s * kChunkRows);
        while (c + 1 < ncolors && r >= c_row0[c + 1]) ++c;
        const int bucket = std::min(7, static_cast<int>(8LL * (r - c_row0[c]) / std::max(1, c_rows[c])));
        key[s] = (static_cast<long long>(bucket) << 40) | (static_cast<long long>(c) << 32) | s;
    }
    std::vector<int> order(ns);
    for (int s = 0; s < ns; ++s) order[s] = s;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return key[a] < key[b]; });
    return order;
}

int build_sell(int n, const int *rowptr, const int *col, const double *val, const int *block_ptr,
               int ncolors, const int *color_ptr, SellMatrix &out) {
    const int ns = (n + kChunkRows - 1) / kChunkRows;
    out.slice_off.assign(ns, 0);
    out.slice_width.assign(ns, 0);
    long long total = 0;
    for (int s = 0; s < ns; ++s) {
        int w = 0;
        for (int i = s * kChunkRows; i < std::min(n, (s + 1) * kChunkRows); ++i)
            w = std::max(w, rowptr[i + 1] - rowptr[i]);
        out.slice_off[s] = static_cast<int>(total);
        out.slice_width[s] = w;
        total += static_cast<long long>(w) * kChunkRows;
        if (total >= (1LL << 31)) return set_error(ICCG_EINVAL, "sliced ELL copy exceeds 2^31 slots");
    }
    out.col.assign(total, -1);
    out.val.assign(total, 0.0);
    for (int s = 0; s < ns; ++s)
        for (int i = s * kChunkRows; i < std::min(n, (s + 1) * kChunkRows); ++i) {
            const int t = i - s * kChunkRows;
            for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                const long long slot = out.slice_off[s] + static_cast<long long>(k - rowptr[i]) * kChunkRows + t;
                out.col[slot] = col[k];
                out.val[slot] = val[k];
            }
        }
    out.order = slice_launch_order(n, ns, block_ptr, ncolors, color_ptr);
    return ICCG_OK;
}

// Row-by-row IC(0): for every k < i in the pattern of row i (ascending),
//   L_ik = (a_ik - sum_j L_ij L_kj) / L_kk   over j < k in both patterns,
// then L_ii = sqrt(a_ii - sum_k L_ik^2).  Row i's finished values are
// scattered into a position map so the inner sum walks row k only.
int ic0_host(int n, const int *rowptr, const int *col, const double *val, const int *dpos,
             std::vector<double> &lval) {
    lval.assign(static_cast<size_t>(rowptr[n]), 0.0);
    std::vector<int> where(n, -1);
    for (int i = 0; i < n; ++i) {
        const int d = dpos[i];
        for (int p = rowptr[i]; p < d; ++p) where[col[p]] = p;
        double pivot = val[d];
        for (int p = rowptr[i]; p < d; ++p) {
            const int k = col[p];
            double s = val[p];
            for (int q = rowptr[k]; q < dpos[k]; ++q) {
                const int w = where[col[q]];
                if (w >= 0) s -= lval[w] * lval[q];
            }
            lval[p] = s / lval[dpos[k]];
        }
        for (int p = rowptr[i]; p < d; ++p) pivot -= lval[p] * lval[p];
        for (int p = rowptr[i]; p < d; ++p) where[col[p]] = -1;
        if (!(pivot > 0.0) || !std::isfinite(pivot)) return i;
        lval[d] = std::sqrt(pivot);
    }
    return -1;
}

}  // namespace iccg
