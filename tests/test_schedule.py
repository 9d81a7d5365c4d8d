"""CPU tests of the substitution schedules libiccg.so builds at setup
(iccg_schedule_stats: host only, no device).

The library re-derives every invariant of both schedules itself (chunks tile
the colors, per-row slot groups, dependencies at earlier colors and launch
positions, rows read across chunks are waited for, remote reads are
exported); these tests run that check over several orderings and packings,
and pin the counts against an independent replica of the packing rules
written here from Algorithm 1's structure (blocks of a color are packed in
order into chunks of at most pack_rows rows; a block larger than 64 rows is
cut into 64-row chunks that one task runs in order)."""
import numpy as np
import pytest

import synth
from paper_2609_00561_amd import iccg


def _replica(rp, cl, bp, cp, forward, pack=64):
    """Independent counts: tasks, chunks, slots, max depth, max width, deps."""
    rp, cl = np.asarray(rp), np.asarray(cl)
    n = rp.size - 1
    chunks, task_chunks = [], []
    for c in range(cp.size - 1):
        cur = None
        for b in range(cp[c], cp[c + 1]):
            r0, r1 = int(bp[b]), int(bp[b + 1])
            if r1 - r0 > 64:
                if cur is not None:
                    task_chunks.append([len(chunks)])
                    chunks.append(tuple(cur))
                    cur = None
                ids = []
                for r in range(r0, r1, 64):
                    ids.append(len(chunks))
                    chunks.append((r, min(r + 64, r1)))
                task_chunks.append(ids)
            else:
                if cur is not None and (cur[1] - cur[0]) + (r1 - r0) > pack:
                    task_chunks.append([len(chunks)])
                    chunks.append(tuple(cur))
                    cur = None
                cur = [r0, r1] if cur is None else [cur[0], r1]
        if cur is not None:
            task_chunks.append([len(chunks)])
            chunks.append(tuple(cur))
    task_of_row = np.empty(n, dtype=np.int64)
    for t, ids in enumerate(task_chunks):
        for ch in ids:
            task_of_row[chunks[ch][0]:chunks[ch][1]] = t
    slots, max_depth, max_width, padded = 0, 0, 0, 0
    for r0, r1 in chunks:
        width, widths, level = 0, 0, {}
        rows = range(r0, r1) if forward else range(r1 - 1, r0 - 1, -1)
        for i in rows:
            js = [int(j) for j in cl[rp[i]:rp[i + 1]] if (j < i if forward else j > i)]
            width = max(width, len(js))
            widths += len(js)
            lev = 0
            for j in js:
                if r0 <= j < r1:
                    lev = max(lev, level[j] + 1)
            level[i] = lev
        slots += width * (r1 - r0) if width > 8 else widths
        padded += width > 8
        max_width = max(max_width, width)
        max_depth = max(max_depth, max(level.values()) + 1)
    rows = np.repeat(np.arange(n), np.diff(rp))
    side = cl < rows if forward else cl > rows
    ti, tj = task_of_row[rows[side]], task_of_row[cl[side]]
    other = ti != tj
    deps = np.unique(ti[other] * len(task_chunks) + tj[other]).size
    return {"tasks": len(task_chunks), "chunks": len(chunks), "slots": slots,
            "max_depth": max_depth, "max_width": max_width, "deps": deps,
            "padded_chunks": padded}


CASES = [
    ("laplace2d_64", "abmc", 64, 64),
    ("poisson7_16", "abmc", 8, 64),
    ("poisson7_16", "abmc", 8, 16),
    ("poisson7_16", "abmc", 8, 1),
    ("poisson7_16", "leiden", ("modularity", 1.0), 64),    # blocks > 64 rows
    ("knn13_20k", "leiden", ("cpm", 0.05), 64),
    ("stencil27_12", "abmc", 32, 64),
    ("poisson7_32", "abmc", 16, 32),
    ("randspd_2k", "abmc", 16, 64),                         # rows of 40-80 entries
    ("randspd6_2k", "abmc", 16, 64),                        # rows of 9-16 entries
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-{c[1]}-{c[2]}-p{c[3]}")
def test_schedule_counts_and_invariants(case):
    name, kind, param, pack = case
    A, _ = synth.workload(name)
    o = iccg.iccg_order_abmc(A, param) if kind == "abmc" else iccg.iccg_order_leiden(A, *param)
    rp, cl, vl = iccg.iccg_permute(A, o.perm)
    got = iccg.iccg_schedule_stats(rp, cl, vl, o.block_ptr, o.color_ptr, pack_rows=pack)
    for d, fwd in (("forward", True), ("backward", False)):
        want = _replica(rp, cl, np.asarray(o.block_ptr), np.asarray(o.color_ptr), fwd, pack)
        for key, v in want.items():
            assert got[d][key] == v, (d, key, got[d][key], v)
        assert got[d]["remote_tasks"] <= got[d]["tasks"]
        assert got[d]["exported_rows"] <= A.n
    # both slot layouts are exercised: the 7-point and 5-point matrices have
    # no chunk wider than 8 entries, the others have padded chunks, and the
    # dense random matrix has rows wider than the 32 entries kept in registers
    if name.startswith(("poisson7", "laplace2d")):
        assert got["forward"]["padded_chunks"] == got["backward"]["padded_chunks"] == 0
    else:
        assert got["forward"]["padded_chunks"] > 0 and got["backward"]["padded_chunks"] > 0
    if name == "randspd_2k":
        assert got["forward"]["padded_chunks"] < got["forward"]["chunks"]
        assert got["forward"]["max_width"] > 32
    if name == "randspd6_2k":
        # the register tier of 16 slots: widest rows between 9 and 16
        assert 8 < got["forward"]["max_width"] <= 16 and 8 < got["backward"]["max_width"] <= 16
    # the two triangles hold the same number of entries, so only padding
    # can differ between the directions
    nnz_l = (A.nnz - A.n) // 2
    assert got["forward"]["slots"] >= nnz_l and got["backward"]["slots"] >= nnz_l


def test_schedule_padding_7point_128():
    """Slot layout of the 7-point 128^3 Poisson matrix under ABMC s = 16: rows
    have at most 6 entries per triangle, so every chunk is stored without
    padding (each row padded to its chunk's widest would hold 1.73x and
    1.78x the entries)."""
    A, _ = synth.workload("poisson7_128")
    o = iccg.iccg_order_abmc(A, 16)
    rp, cl, vl = iccg.iccg_permute(A, o.perm)
    got = iccg.iccg_schedule_stats(rp, cl, vl, o.block_ptr, o.color_ptr)
    nnz_l = (A.nnz - A.n) // 2
    assert got["forward"]["slots"] == nnz_l == 6242304 and got["backward"]["slots"] == nnz_l
    assert got["forward"]["tasks"] == 32772 and got["forward"]["max_width"] == 6


def test_schedule_random_graphs():
    rng = np.random.default_rng(5)
    for trial in range(10):
        n = int(rng.integers(2, 400))
        A = synth.random_spd_mmatrix(n, float(rng.uniform(0.01, 0.2)), rng)
        for s in (1, 5, 70):
            o = iccg.iccg_order_abmc(A, s)
            rp, cl, vl = iccg.iccg_permute(A, o.perm)
            got = iccg.iccg_schedule_stats(rp, cl, vl, o.block_ptr, o.color_ptr)
            want = _replica(rp, cl, np.asarray(o.block_ptr), np.asarray(o.color_ptr), True)
            assert got["forward"]["tasks"] == want["tasks"], (trial, s)
            assert got["forward"]["deps"] == want["deps"], (trial, s)


def test_schedule_stats_rejects_bad_ordering():
    A, _ = synth.workload("laplace2d_64")
    o = iccg.iccg_order_abmc(A, 64)
    rp, cl, vl = iccg.iccg_permute(A, o.perm)
    with pytest.raises(iccg.IccgError) as e:
        iccg.iccg_schedule_stats(rp, cl, vl, o.block_ptr, np.array([0, o.nblocks]))
    assert e.value.status == iccg.ICCG_EBADORDER
