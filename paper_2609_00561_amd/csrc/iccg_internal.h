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
    int16_t nrows;   // 1..64
    int16_t width;   // max entries of a row in this chunk
    int16_t depth;   // number of intra-chunk levels (>= 1)
    int16_t pad;
};
static_assert(sizeof(Chunk) == 16, "Chunk layout");

// Per-row schedule word: number of entries whose value is final before the
// chunk starts (bits 0..15), number of entries inside the chunk (bits
// 16..23), intra-chunk level (bits 24..31).  The row's entries are stored
// "before-chunk first", each group in ascending column order.
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
    std::vector<Chunk> chunks;
    std::vector<uint32_t> meta;        // n
    std::vector<int> slot_col;         // column per slot, -1 for padding
    std::vector<int> slot_src;         // CSR position of the factor value, -1 for padding
    int max_depth = 0;
};

// Builds both sweep plans from the validated permuted pattern.  tpos[k] is
// the CSR position of the transpose of entry k.
int build_sweep_plan(bool forward, int n, const int *rowptr, const int *col, const int *tpos,
                     int nblocks, const int *block_ptr, int ncolors, const int *color_ptr,
                     int pack_rows, SweepPlan &out);

// Host FP64 IC(0) on the CSR pattern; lval gets A's positions (upper part 0).
// Returns -1 or the first row whose pivot is not > 0 or not finite.
int ic0_host(int n, const int *rowptr, const int *col, const double *val, const int *dpos,
             std::vector<double> &lval);

}  // namespace iccg
