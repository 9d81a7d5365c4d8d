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
// one 64-row piece of a block larger than 64 rows.  Its sweep entries are
// stored slot-major: entry k of the chunk's row t sits at off + k*nrows + t,
// so the lanes of a wavefront read consecutive addresses.
struct Chunk {
    int32_t row0;    // first row (permuted numbering)
    int32_t off;     // first slot of this chunk
    int32_t shape;   // nrows (1..64) | width << 16 (max entries of a row)
    int32_t depth;   // number of intra-chunk levels (>= 1)
    int nrows() const { return shape & 0xffff; }
    int width() const { return shape >> 16; }
};
static_assert(sizeof(Chunk) == 16, "Chunk layout");

// One wavefront task: its first chunk in processing order (forward: lowest,
// backward: highest) inline, so a task starts from a single 32-byte load, the
// range [c0, c1) of all its chunks and, for the single-launch sweep, its
// dependency list deps[dep0, dep0 + ndeps) and kind bits.
struct TaskRec {
    Chunk first;
    int32_t c0, c1;
    int32_t dep0;
    int32_t kind_ndeps;   // kTaskRemote | kTaskExports | ndeps << 2
    int nchunks() const { return c1 - c0; }
};
static_assert(sizeof(TaskRec) == 32, "TaskRec layout");

// Per-row schedule word: number of entries whose value is final before the
// chunk starts (bits 0..14), the export bit (bit 15, see kMetaExport),
// number of entries inside the chunk (bits 16..23), intra-chunk level (bits
// 24..31).  The row's entries are stored "before-chunk first", each group in
// ascending column order.
constexpr uint32_t kMetaNextMask = 0x7fffu;
// Single-launch sweep: the row is read by a task of another region (or by a
// task that reads through device-coherent loads), so its value is also
// written through to memory.
constexpr uint32_t kMetaExport = 0x8000u;
// TaskRec.kind bits of the single-launch sweep.
constexpr int kTaskRemote = 1;   // some dependency is in another region
constexpr int kTaskExports = 2;  // some row of the task has kMetaExport
inline uint32_t pack_meta(int n_ext, int n_int, int level) {
    return static_cast<uint32_t>(n_ext) | (static_cast<uint32_t>(n_int) << 16) |
           (static_cast<uint32_t>(level) << 24);
}

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
    std::vector<int> slot_col;         // column per slot, -1 for padding
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
