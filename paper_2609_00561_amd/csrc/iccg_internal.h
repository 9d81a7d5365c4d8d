// Internal declarations shared by the host setup code and the HIP sources of
// libiccg.so.  Not part of the public ABI (that is include/iccg.h).
#pragma once

#include "iccg.h"

#include <cstdint>
#include <string>
#include <vector>

namespace iccg {

// Records a message for iccg_last_error() and returns code.
int set_error(int code, const std::string &msg);

// Rows handled by one wavefront at a time (one lane per row).
constexpr int kChunkRows = 64;

// A chunk is up to 64 consecutive rows of one color that one wavefront
// substitutes together: either several whole blocks packed side by side or
// one 64-row piece of a block larger than 64 rows.  Its rows are given
// "sorted positions" by decreasing number of entries (ties by row), and its
// sweep entries are stored slot-major over those positions as jagged
// diagonals: slot k holds entry k of the cnt_k rows that have more than k
// entries, the row at sorted position l at off + cnt_0 + ... + cnt_{k-1} + l.
// So the lanes of a wavefront read consecutive addresses and no padding is
// stored.  A chunk whose widest row has more than kJaggedMaxWidth entries is
// padded instead: every row is stored at its own position for each of the
// width slots (cnt_k = nrows, sorted position = row position, empty slots hold
// column -1 and value 0).
constexpr int kJaggedMaxWidth = 8;
struct Chunk {
    int32_t row0;    // first row (permuted numbering)
    int32_t off;     // first slot of this chunk
    int32_t shape;   // nrows (1..64) | width << 16 (max entries of a row)
    int32_t depth;   // number of intra-chunk levels (>= 1)
    uint32_t cnt[2]; // jagged chunks: cnt_k in byte k (k < width); else 0
    int32_t pad[2];
    int nrows() const { return shape & 0xffff; }
    int width() const { return shape >> 16; }
    bool jagged() const { return width() <= kJaggedMaxWidth; }
    int slot_rows(int k) const { return jagged() ? static_cast<int>((cnt[k >> 2] >> (8 * (k & 3))) & 0xffu) : nrows(); }
};
static_assert(sizeof(Chunk) == 32, "Chunk layout");

// One wavefront task: its first chunk in processing order (forward: lowest,
// backward: highest) inline, so a task starts from a single 64-byte load, the
// range [c0, c1) of all its chunks and, for the single-launch sweep, its
// dependency list deps[dep0, dep0 + ndeps) and kind bits.
struct TaskRec {
    Chunk first;
    int32_t c0, c1;
    int32_t dep0;
    int32_t kind_ndeps;   // kTaskRemote | kTaskExports | ndeps << 2
    int32_t wide;         // index among the wide tasks (see WidePlan), or -1
    int32_t pad[3];
    int nchunks() const { return c1 - c0; }
};
static_assert(sizeof(TaskRec) == 64, "TaskRec layout");

// Per-row schedule word: number of entries whose value is final before the
// chunk starts (bits 0..12), the export bit (bit 13, see kMetaExport), the
// row's sorted position in its chunk (bits 14..19), number of entries inside
// the chunk (bits 20..25), intra-chunk level (bits 26..31).  The row's entries
// are stored "before-chunk first", each group in ascending column order.
constexpr uint32_t kMetaNextMask = 0x1fffu;
// Single-launch sweep: the row is read by a task of another region (or by a
// task that reads through device-coherent loads), so its value is also
// written through to memory.
constexpr uint32_t kMetaExport = 0x2000u;
constexpr int kMetaPosShift = 14;
constexpr int kMetaInnerShift = 20;
constexpr int kMetaLevelShift = 26;
// TaskRec.kind bits of the single-launch sweep.
constexpr int kTaskRemote = 1;   // some dependency is in another region
constexpr int kTaskExports = 2;  // some row of the task has kMetaExport
inline uint32_t pack_meta(int n_ext, int n_int, int level, int pos) {
    return static_cast<uint32_t>(n_ext) | (static_cast<uint32_t>(pos) << kMetaPosShift) |
           (static_cast<uint32_t>(n_int) << kMetaInnerShift) |
           (static_cast<uint32_t>(level) << kMetaLevelShift);
}
inline int meta_next(uint32_t m) { return static_cast<int>(m & kMetaNextMask); }
inline int meta_pos(uint32_t m) { return static_cast<int>((m >> kMetaPosShift) & 63u); }
inline int meta_inner(uint32_t m) { return static_cast<int>((m >> kMetaInnerShift) & 63u); }
inline int meta_level(uint32_t m) { return static_cast<int>(m >> kMetaLevelShift); }

// One sweep direction.  Forward: row i uses L_ij, j < i; chunks of a task run
// in ascending order, colors ascending.  Backward: row i uses (L^T)_ij = L_ji,
// j > i; chunks of a task run in descending order, colors descending.
struct SweepPlan {
    bool forward = true;
    std::vector<int> color_task_ptr;   // ncolors+1, tasks of each color
    std::vector<int> task_chunk_ptr;   // ntasks+1
    std::vector<TaskRec> tasks;        // ntasks
    std::vector<Chunk> chunks;
    std::vector<uint32_t> meta;        // n
    std::vector<int> slot_col;         // column per slot, -1 for padding (see Chunk)
    std::vector<int> slot_src;         // CSR position of the factor value, -1 for padding
    int max_depth = 0;
    int max_width = 0;
    // tasks of other colors whose rows this task reads (dependency lists for
    // the single-launch sweep); all are earlier in the sweep's processing order
    std::vector<int> dep_ptr;          // ntasks+1
    std::vector<int> deps;
    // launch table of the single-launch sweep: workgroup b runs task wg_task[b].
    // Workgroups follow the processing order color by color; inside a color,
    // the workgroups dealt to one XCD (b mod 8) get one contiguous region of
    // the color's tasks, the same region of the domain in every color.
    std::vector<int> wg_task;
    long long remote_tasks = 0;        // tasks with kTaskRemote
    long long exported_rows = 0;       // rows with kMetaExport
};

// Wide tasks (per-color launches only).  A task that is one block of more
// than kWideMinRows rows would otherwise run its 64-row chunks one after
// another on one wavefront.  Instead a workgroup of wide_waves(width)
// wavefronts runs it in pieces of 64 rows per wavefront, in the sweep's
// processing order; each piece gets a level schedule over all of its rows, so
// a level's rows anywhere in the piece run together.  Per row: entries outside the piece first, then those inside
// it, each group ascending; the piece's rows are stored as 64-row sub-chunks
// in the padded slot layout.
// Wavefronts per wide workgroup: 16 when every row of the schedule has at
// most 8 entries (the kernel's registers then allow 16 wavefronts on a
// compute unit), else 8.
constexpr int wide_waves(int max_width) { return max_width <= 8 ? 16 : 8; }
constexpr int kWideMaxRows = 64 * 16;
// Smaller multi-chunk blocks stay on one wavefront: for a few chunks the
// workgroup's barriers cost more than the sequence (measured on blocks of
// 65-67 rows).
constexpr int kWideMinRows = 256;
struct WidePiece {
    int32_t sub0, nsub;   // sub-chunks [sub0, sub0 + nsub) of WidePlan::subs
    int32_t depth;        // levels of the piece
    int32_t row0;         // first row of the piece
};
struct WidePlan {
    std::vector<int> color_ptr;      // ncolors+1: wide tasks of each color
    std::vector<int> task;           // task id of each wide task
    std::vector<int> piece_ptr;      // nwide+1: pieces of each wide task, in processing order
    std::vector<WidePiece> pieces;
    std::vector<Chunk> subs;         // row0, off, shape (nrows | width << 16) of each sub-chunk
    std::vector<uint32_t> wmeta;     // n: entries outside | entries inside << 16 (rows of wide tasks)
    std::vector<int> wlev;           // n: level inside the piece
    std::vector<int> slot_col, slot_src;
    int max_depth = 0;
};
// Marks the tasks of plan that are single blocks of more than kWideMinRows
// rows as wide and builds their pieces.  An empty WidePlan (no wide task) is
// valid.
int build_wide_plan(SweepPlan &plan, int n, const int *rowptr, const int *col, const int *tpos,
                    int ncolors, int piece_rows, WidePlan &out);

// Sliced ELL copy of A' for the SpMV: slices of 64 consecutive rows; entry k
// of the slice's row t at slice_off[s] + k*64 + t (column -1, value 0 pads).
struct SellMatrix {
    std::vector<int> slice_off, slice_width;   // nslices
    std::vector<int> order;                    // launch order of the slices (see build_sell)
    std::vector<int> col;
    std::vector<double> val;
};
int build_sell(int n, const int *rowptr, const int *col, const double *val, const int *block_ptr,
               int ncolors, const int *color_ptr, SellMatrix &out);

// Builds both sweep plans from the validated permuted pattern.  tpos[k] is
// the CSR position of the transpose of entry k.
int check_sweep_plan(const SweepPlan &plan, int n, const int *rowptr, const int *col, int ncolors,
                     const int *block_ptr, const int *color_ptr);
int build_sweep_plan(bool forward, int n, const int *rowptr, const int *col, const int *tpos,
                     int nblocks, const int *block_ptr, int ncolors, const int *color_ptr,
                     int pack_rows, SweepPlan &out);

// Host FP64 IC(0) on the CSR pattern; lval gets A's positions (upper part 0).
// Returns -1 or the first row whose pivot is not > 0 or not finite.
int ic0_host(int n, const int *rowptr, const int *col, const double *val, const int *dpos,
             std::vector<double> &lval);

}  // namespace iccg
