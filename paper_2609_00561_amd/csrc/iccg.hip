// MI355X (gfx950) device path of block-multicolored ICCG and the C ABI in
// include/iccg.h.
//
// Per CG iteration k (Section 5, IC(0)-preconditioned CG):
//   x += alpha_{k-1} p_{k-1}, p = z + beta p  k_update_p (the x update of the
//                                             previous iteration, deferred)
//   q = A'p with (p, q)                       k_spmv
//   alpha = (r, z)/(p, q)                     k_reduce
//   r -= alpha q, ||r||^2 per task,
//   y = L^{-1} r   (Algorithm 1)              k_sweep<forward>, one launch per color
//   z = L^{-T} y, (r, z) per task             k_sweep<backward>, one launch per color
// (or, by option, k_sweep_flow: one dataflow launch for all colors, or for
// the small ones only)
//   stopping test on ||r||, beta, rho         k_reduce_rr_beta
// (inside the loop the last color of both sweeps runs as one k_sweep_turn
// launch: its forward then its backward substitution, task by task)
// and after the last iteration x += alpha p   k_axpy_alpha
// The sweeps give every 64-row chunk of a color one wavefront (one lane per
// row): the terms whose values were final before the chunk started are
// gathered by all lanes at once, the in-chunk terms follow the chunk's level
// schedule through LDS.  Every row computes the same terms as the serial sweep.
//
// All reductions are two-pass and deterministic: a fixed tree inside each
// workgroup, then one workgroup sums the partials in index order.
//
// A device-side flag stops the work of every kernel once the stopping test has
// passed, so batches of iterations can be queued (and replayed as one HIP
// graph) with a single host read of the flag per batch.
#include <hip/hip_runtime.h>

#include "iccg_device.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

namespace iccg {

thread_local std::string g_last_error;

int set_error(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

}  // namespace iccg

using namespace iccg;

enum ReduceOp : int {
    OP_STORE = 0,    // out[0] = sum
    OP_BNORM = 1,    // bnorm = sqrt(sum)
    OP_INIT_RR = 2,  // relres = sqrt(sum)/bnorm, hist[0], stopping test
    OP_RHO = 3,      // rho = sum
    OP_ALPHA = 4,    // alpha = rho / sum (sum = (p, q))
    OP_RR = 5,       // iteration done: iter++, relres, hist, stopping test
    OP_BETA = 6,     // beta = sum / rho, rho = sum
    OP_TRUE = 7,     // relres_true = sqrt(sum)/bnorm
};

constexpr int kVecThreads = 256;
constexpr int kReduceThreads = 1024;
constexpr int kMaxVecBlocks = 2048;   // multiple of 8

// Workgroups are dealt to the 8 XCDs round robin; give each XCD one
// contiguous range of logical blocks so neighbouring rows share an L2.
// A bijection on [0, G).
__device__ inline int xcd_remap(int b, int G) {
    const int x = b & 7, i = b >> 3;
    const int q = G >> 3, r = G & 7;
    return x * q + min(x, r) + i;
}

// The stopping flag a launch tests before its work: the solve's, or, for a
// launch outside a solve (no scalar block), one that always reads
// DONE_RUNNING.  Reading it through a selected pointer keeps the load free of
// a branch, so it is issued together with the launch's first other loads and
// the launch waits for one memory round trip, not two in a row.
__device__ int g_running = DONE_RUNNING;   // never written
__device__ __forceinline__ const int *done_flag(const DevScalars *sc) {
    return sc ? &sc->done : &g_running;
}

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
    // fixed butterfly over the 64 lanes of a wavefront
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic sum over a workgroup of NT threads; result valid in thread 0.
template <int NT>
__device__ inline double block_sum(double v) {
    __shared__ double red[NT / 64];
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < NT / 64; ++k) s += red[k];
    return s;
}

// Thread t's share of a fixed-order sum over part[0, np): pairs (2i, 2i+1)
// for i = t, t + NT, ... in that order, loaded 16 bytes at a time with up to
// kPartialRound pairs in flight, so one workgroup of 1024 threads covers 40K
// partials in one round trip (a sweep's 32K tasks and a few more: 16 pairs
// per thread left the last handful of partials to a second round trip).
constexpr int kPartialRound = 20;
template <int NT>
__device__ __forceinline__ double thread_partial(const double *__restrict__ part, int np) {
    const int npair = np >> 1;
    const double2 *p2 = reinterpret_cast<const double2 *>(part);
    double v = 0.0;
    for (int base = 0; base < npair; base += kPartialRound * NT) {
        double2 buf[kPartialRound];
#pragma unroll
        for (int u = 0; u < kPartialRound; ++u) {
            const int i = base + u * NT + static_cast<int>(threadIdx.x);
            buf[u] = i < npair ? p2[i] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < kPartialRound; ++u) v += buf[u].x + buf[u].y;
    }
    if ((np & 1) && threadIdx.x == 0) v += part[np - 1];
    return v;
}

// One workgroup per column of a block of right-hand sides (one for a single
// vector): column c reduces part[c * part_ld ...] into its scalars sc[c].
__global__ __launch_bounds__(kReduceThreads) void k_reduce(const double *__restrict__ part,
                                                           int np, DevScalars *sc, int op,
                                                           double *__restrict__ out,
                                                           double *__restrict__ hist, int part_ld,
                                                           int hist_ld) {
    const int col = blockIdx.x;
    part += static_cast<size_t>(col) * part_ld;
    sc += col;
    hist += static_cast<size_t>(col) * hist_ld;
    if (out) out += col;
    // the stopping flag is read together with the partials and tested after
    // the sum (only thread 0 writes), so the launch waits for one round trip
    const bool stopped = sc->done != DONE_RUNNING;
    double v = thread_partial<kReduceThreads>(part, np);
    v = block_sum<kReduceThreads>(v);
    if (threadIdx.x != 0) return;
    if (op != OP_STORE && op != OP_TRUE && op != OP_BNORM && stopped) return;
    switch (op) {
        case OP_STORE: out[0] = v; break;
        case OP_BNORM: sc->bnorm = (v > 0.0) ? sqrt(v) : 1.0; break;
        case OP_INIT_RR: {
            const double rel = sqrt(v) / sc->bnorm;
            sc->relres = rel;
            if (sc->hist_cap > 0) hist[0] = rel;
            if (rel <= sc->tol) sc->done = DONE_CONVERGED;
            else if (!isfinite(rel)) sc->done = DONE_NAN;
            else if (sc->maxit <= 0) sc->done = DONE_MAXIT;
            break;
        }
        case OP_RHO:
            sc->rho = v;
            if (!isfinite(v)) sc->done = DONE_NAN;
            break;
        case OP_ALPHA:
            if (!(v > 0.0) || !isfinite(v)) { sc->done = DONE_NAN; break; }
            sc->alpha = sc->rho / v;
            break;
        case OP_RR: {
            const int it = sc->iter + 1;
            sc->iter = it;
            const double rel = sqrt(v) / sc->bnorm;
            sc->relres = rel;
            if (it < sc->hist_cap) hist[it] = rel;
            if (rel <= sc->tol) sc->done = DONE_CONVERGED;
            else if (!isfinite(rel)) sc->done = DONE_NAN;
            else if (it >= sc->maxit) sc->done = DONE_MAXIT;
            break;
        }
        case OP_BETA:
            if (!isfinite(v)) { sc->done = DONE_NAN; break; }
            sc->beta = v / sc->rho;
            sc->rho = v;
            break;
        case OP_TRUE: sc->relres_true = sqrt(v) / sc->bnorm; break;
    }
}

// End of a CG iteration in one launch: ||r||^2 from the forward sweep's
// partials decides the stopping test (as OP_RR), then, if the iteration goes
// on, (r, z) from the backward sweep's partials gives beta (as OP_BETA).  The
// backward sweep does not depend on the stopping test, so it can run first;
// after the last iteration its z is simply unused.  Same sums, same order as
// two k_reduce launches.
// (one workgroup per column of a block of right-hand sides, as k_reduce)
__global__ __launch_bounds__(kReduceThreads) void k_reduce_rr_beta(const double *__restrict__ rr_part,
                                                                   int n_rr,
                                                                   const double *__restrict__ rz_part,
                                                                   int n_rz, DevScalars *sc,
                                                                   double *__restrict__ hist, int part_ld,
                                                                   int hist_ld) {
    const int col = blockIdx.x;
    rr_part += static_cast<size_t>(col) * part_ld;
    rz_part += static_cast<size_t>(col) * part_ld;
    sc += col;
    hist += static_cast<size_t>(col) * hist_ld;
    // stopping flag read together with the partials, tested by thread 0
    const bool stopped = sc->done != DONE_RUNNING;
    double a = thread_partial<kReduceThreads>(rr_part, n_rr);
    double b = thread_partial<kReduceThreads>(rz_part, n_rz);
    a = block_sum<kReduceThreads>(a);
    __syncthreads();   // block_sum's scratch is reused
    b = block_sum<kReduceThreads>(b);
    if (threadIdx.x != 0 || stopped) return;
    const int it = sc->iter + 1;
    sc->iter = it;
    const double rel = sqrt(a) / sc->bnorm;
    sc->relres = rel;
    if (it < sc->hist_cap) hist[it] = rel;
    if (rel <= sc->tol) { sc->done = DONE_CONVERGED; return; }
    if (!isfinite(rel)) { sc->done = DONE_NAN; return; }
    if (it >= sc->maxit) { sc->done = DONE_MAXIT; return; }
    if (!isfinite(b)) { sc->done = DONE_NAN; return; }
    sc->beta = b / sc->rho;
    sc->rho = b;
}

// one workgroup per column
__global__ void k_init_scalars(DevScalars *sc, double tol, int maxit, int hist_cap) {
    sc += blockIdx.x;
    if (threadIdx.x == 0) {
        sc->rho = sc->alpha = sc->beta = 0.0;
        sc->bnorm = 1.0;
        sc->relres = sc->relres_true = 0.0;
        sc->tol = tol;
        sc->iter = 0;
        sc->done = DONE_RUNNING;
        sc->maxit = maxit;
        sc->hist_cap = hist_cap;
    }
}

// ---------------------------------------------------------------------------
// SpMV on the sliced ELL copy (one wavefront per 64-row slice, one lane per row)
//   SP_PLAIN: y = A x, partial (x, y)
//   SP_RESID: y = b - A x, partial (y, y)
// ---------------------------------------------------------------------------
enum SpmvMode : int { SP_PLAIN = 0, SP_RESID = 1 };
// Slices per wavefront: two for rows of up to 8 entries; one for wider rows,
// whose WMAX slots per slice already keep enough loads in flight and whose
// registers for two slices would leave one wavefront per SIMD (WMAX = 32).
constexpr int spmv_slices_per_wave(int wmax) { return wmax <= 8 ? 2 : 1; }
constexpr int kSpmvMaxSlicesPerWave = 2;
template <int U>
struct alignas(16 * U) SliceRecs {
    int4 r[U];
};
// Columns (wavefronts) per workgroup of the block-of-right-hand-sides kernels.
constexpr int kColWaves = 8;

// One wavefront per U = spmv_slices_per_wave(WMAX) consecutive launch
// positions (the grid has ceil(nslices / U) wavefronts); the slots of a row
// are taken in rounds of up to 16 (loads in registers at once, then the
// gathers, then the terms), the row sum in ascending column order.  wg: the
// wavefront's logical index; lane 0
// writes the wavefront's partial sum to *part_out.  NT: stream the matrix
// with non-temporal loads.  stop: the solve's stopping flag (the wavefront
// returns at once unless it reads DONE_RUNNING).
template <int MODE, int WMAX, bool NT>
__device__ __forceinline__ void spmv_wave(int n, int nslices, const int4 *__restrict__ slices,
                                          const int *__restrict__ col, const double *__restrict__ val,
                                          const double *__restrict__ x, double *__restrict__ y,
                                          const double *__restrict__ b, double *__restrict__ part_out,
                                          int wg, const int *stop) {
    constexpr int U = spmv_slices_per_wave(WMAX);
    const int lane = static_cast<int>(threadIdx.x) & 63;
    const int lg0 = wg * U;
    // U consecutive launch positions at once, so one wavefront has all of
    // their loads in flight together.  Launch-ordered slice record:
    // (slice, first slot, width), padded to a whole number of wavefronts
    // with empty records.  The records and the stopping flag are loaded
    // together, so the wavefront waits for one memory round trip before its
    // matrix loads; a stopped solve leaves every slice with no rows and no
    // slots, and then nothing else is loaded or stored but the partial sum
    // (zero).
    const SliceRecs<U> recs = reinterpret_cast<const SliceRecs<U> *>(slices)[wg];
    const bool running = *stop == DONE_RUNNING;
    int off[U], w[U], row[U];
    double own_x[U], own_b[U], sum[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const bool valid = running && lg0 + u < nslices;
        const int4 rec = recs.r[u];
        off[u] = rec.y + lane;
        w[u] = valid ? rec.z : 0;
        row[u] = valid ? rec.x * 64 + lane : n;
        sum[u] = 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        own_x[u] = 0.0;
        own_b[u] = 0.0;
        if (row[u] < n) {
            own_x[u] = x[row[u]];
            if (MODE == SP_RESID) own_b[u] = b[row[u]];
        }
    }
    // Slots in rounds of at most 16 (rows wider than 16 entries take two
    // rounds, so a wavefront holds 16 slots' registers, not 32): every load
    // of a round at once, then its gathers, then its terms in ascending
    // column order.  The matrix streams through once (non-temporal: it
    // should not push the gathered vector out of L2), unless several
    // wavefronts read it.
    constexpr int RS = WMAX < 16 ? WMAX : 16;
#pragma unroll 1
    for (int r0 = 0; r0 < WMAX; r0 += RS) {
        int cc[U][RS];
        double vv[U][RS], xv[U][RS];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < RS; ++j)
                if (r0 + j < w[u]) {
                    const int sl = off[u] + (r0 + j) * 64;
                    if (NT) {
                        cc[u][j] = __builtin_nontemporal_load(col + sl);
                        vv[u][j] = __builtin_nontemporal_load(val + sl);
                    } else {
                        cc[u][j] = col[sl];
                        vv[u][j] = val[sl];
                    }
                }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < RS; ++j)
                if (r0 + j < w[u]) xv[u][j] = x[cc[u][j] < 0 ? 0 : cc[u][j]];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < RS; ++j)
                if (r0 + j < w[u]) sum[u] = (cc[u][j] >= 0) ? sum[u] + vv[u][j] * xv[u][j] : sum[u];
    }
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        for (int k = WMAX; k < w[u]; ++k) {
            const int c = col[off[u] + k * 64];
            if (c >= 0) sum[u] += val[off[u] + k * 64] * x[c];
        }
        if (row[u] < n) {
            if (MODE == SP_PLAIN) {
                y[row[u]] = sum[u];
                acc += own_x[u] * sum[u];
            } else {
                const double rv = own_b[u] - sum[u];
                y[row[u]] = rv;
                acc += rv * rv;
            }
        }
    }
    const double t = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) *part_out = t;
}

// (sc among the leading, preloaded arguments, as for k_sweep)
template <int MODE, int WMAX>
__global__ __launch_bounds__(64) void k_spmv(int n, int nslices, const int4 *__restrict__ slices,
                                             const DevScalars *sc,
                                             const int *__restrict__ col,
                                             const double *__restrict__ val,
                                             const double *__restrict__ x,
                                             double *__restrict__ y,
                                             const double *__restrict__ b,
                                             double *__restrict__ part) {
    // the grid is ceil(nslices / U) (computed here rather than read from the
    // dispatch packet, so the launch's first loads are its own)
    constexpr int U = spmv_slices_per_wave(WMAX);
    const int grid = (nslices + U - 1) / U;
    spmv_wave<MODE, WMAX, true>(n, nslices, slices, col, val, x, y, b, part + blockIdx.x,
                                xcd_remap(blockIdx.x, grid), done_flag(sc));
}

// Block of right-hand sides (columns ld apart): workgroup g runs the slices
// of k_spmv's workgroup g once per column, one wavefront per column (up to
// kColWaves per workgroup, blockIdx.y counts groups of them); the
// matrix comes from HBM once and from the compute unit's caches for the
// other columns, and every column computes exactly what k_spmv computes for
// it.  part[c * part_ld + g]; columns whose solve has stopped
// skip their work.
template <int MODE, int WMAX>
__global__ __launch_bounds__(64 * kColWaves) void k_spmv_cols(int n, int nslices, const int4 *__restrict__ slices,
                                                    const int *__restrict__ col,
                                                    const double *__restrict__ val,
                                                    const double *__restrict__ x,
                                                    double *__restrict__ y,
                                                    const double *__restrict__ b,
                                                    double *__restrict__ part,
                                                    const DevScalars *sc, int ld, int part_ld,
                                                    int ncols) {
    const int c = static_cast<int>(blockIdx.y) * kColWaves +
                  __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    if (c >= ncols) return;
    if (sc && sc[c].done != DONE_RUNNING) return;
    const size_t off = static_cast<size_t>(c) * ld;
    spmv_wave<MODE, WMAX, false>(n, nslices, slices, col, val, x + off, y + off, b ? b + off : nullptr,
                                 part + static_cast<size_t>(c) * part_ld + blockIdx.x,
                                 xcd_remap(blockIdx.x, gridDim.x), done_flag(nullptr));
}

// ---------------------------------------------------------------------------
// BLAS-1 helpers
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kVecThreads) void k_dot(int n, const double *__restrict__ a,
                                                     const double *__restrict__ b,
                                                     double *__restrict__ part) {
    double acc = 0.0;
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    for (int i = wg * kVecThreads + threadIdx.x; i < n; i += gridDim.x * kVecThreads)
        acc += a[i] * b[i];
    const double t = block_sum<kVecThreads>(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(kVecThreads) void k_fill(int n, double *__restrict__ dst, double v) {
    for (int i = blockIdx.x * kVecThreads + threadIdx.x; i < n; i += gridDim.x * kVecThreads)
        dst[i] = v;
}

// x += alpha p (the previous iteration's step, alpha still in the scalar
// block), then p = z + beta p.  alpha = beta = 0 and p = 0 before the first
// iteration.
// One workgroup per slice (the grid has nslices workgroups), visited in the
// SpMV's launch order and XCD mapping, so the p values each XCD writes are
// the ones its SpMV workgroups gather.
__global__ __launch_bounds__(64) void k_update_p(int n, int nslices,
                                                 const int *__restrict__ slice_order,
                                                 double *__restrict__ x, double *__restrict__ p,
                                                 const double *__restrict__ z,
                                                 const DevScalars *sc) {
    // the slice index and the stopping flag are loaded together and tested
    // at once (one memory round trip before the vector loads)
    const int i = slice_order[xcd_remap(blockIdx.x, nslices)] * 64 + static_cast<int>(threadIdx.x);
    const double alpha = sc->alpha, beta = sc->beta;
    if ((sc->done == DONE_RUNNING) & (i < n)) {
        const double pi = p[i];
        x[i] = x[i] + alpha * pi;
        p[i] = z[i] + beta * pi;
    }
}

// x += alpha p once the iterations have stopped at the stopping test: the
// last iteration's step, which no later k_update_p applies.  After a
// breakdown (non-finite or non-positive (p, q), non-finite residual) x keeps
// the last complete iterate.
__global__ __launch_bounds__(kVecThreads) void k_axpy_alpha(int n, double *__restrict__ x,
                                                            const double *__restrict__ p,
                                                            const DevScalars *sc) {
    if (sc->done != DONE_CONVERGED && sc->done != DONE_MAXIT) return;
    const double alpha = sc->alpha;
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    for (int i = wg * kVecThreads + threadIdx.x; i < n; i += gridDim.x * kVecThreads)
        x[i] = x[i] + alpha * p[i];
}

// out_i = sqrt(a'_ii) in_i (the diagonal scaling of the learned form's probes)
__global__ __launch_bounds__(kVecThreads) void k_scale_sqrt_diag(int n, const int *__restrict__ dpos,
                                                                 const double *__restrict__ val,
                                                                 const double *__restrict__ in,
                                                                 double *__restrict__ out) {
    for (int i = blockIdx.x * kVecThreads + threadIdx.x; i < n; i += gridDim.x * kVecThreads)
        out[i] = sqrt(val[dpos[i]]) * in[i];
}

// v *= target / sqrt(*sumsq)
__global__ __launch_bounds__(kVecThreads) void k_rescale_to_norm(int n, double *__restrict__ v,
                                                                 const double *__restrict__ sumsq,
                                                                 double target) {
    const double f = target / sqrt(*sumsq);
    for (int i = blockIdx.x * kVecThreads + threadIdx.x; i < n; i += gridDim.x * kVecThreads)
        v[i] = v[i] * f;
}

// Column versions of the vector kernels for a block of right-hand sides
// (columns ld apart; blockIdx.y = column; same per-element arithmetic and,
// for the dots, the same partial sums per column as the single-vector
// kernels).  Columns whose solve has stopped skip their work.
__global__ __launch_bounds__(kVecThreads) void k_dot_cols(int n, const double *__restrict__ a,
                                                          const double *__restrict__ b,
                                                          double *__restrict__ part, int ld,
                                                          int part_ld) {
    const size_t off = static_cast<size_t>(blockIdx.y) * ld;
    a += off;
    b += off;
    double acc = 0.0;
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    for (int i = wg * kVecThreads + threadIdx.x; i < n; i += gridDim.x * kVecThreads)
        acc += a[i] * b[i];
    const double t = block_sum<kVecThreads>(acc);
    if (threadIdx.x == 0) part[static_cast<size_t>(blockIdx.y) * part_ld + blockIdx.x] = t;
}

__global__ __launch_bounds__(64) void k_update_p_cols(int n, int nslices,
                                                      const int *__restrict__ slice_order,
                                                      double *__restrict__ x, double *__restrict__ p,
                                                      const double *__restrict__ z,
                                                      const DevScalars *sc, int ld) {
    const DevScalars &s = sc[blockIdx.y];
    if (s.done != DONE_RUNNING) return;
    const double alpha = s.alpha, beta = s.beta;
    const size_t off = static_cast<size_t>(blockIdx.y) * ld;
    x += off;
    p += off;
    z += off;
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    for (int lg = wg; lg < nslices; lg += gridDim.x) {
        const int i = slice_order[lg] * 64 + static_cast<int>(threadIdx.x);
        if (i < n) {
            const double pi = p[i];
            x[i] = x[i] + alpha * pi;
            p[i] = z[i] + beta * pi;
        }
    }
}

__global__ __launch_bounds__(kVecThreads) void k_axpy_alpha_cols(int n, double *__restrict__ x,
                                                                 const double *__restrict__ p,
                                                                 const DevScalars *sc, int ld) {
    const DevScalars &s = sc[blockIdx.y];
    if (s.done != DONE_CONVERGED && s.done != DONE_MAXIT) return;
    const double alpha = s.alpha;
    const size_t off = static_cast<size_t>(blockIdx.y) * ld;
    x += off;
    p += off;
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    for (int i = wg * kVecThreads + threadIdx.x; i < n; i += gridDim.x * kVecThreads)
        x[i] = x[i] + alpha * p[i];
}

template <typename A, typename B>
__global__ __launch_bounds__(kVecThreads) void k_convert(int n, A *__restrict__ dst,
                                                         const B *__restrict__ src) {
    for (int i = blockIdx.x * kVecThreads + threadIdx.x; i < n; i += gridDim.x * kVecThreads)
        dst[i] = static_cast<A>(src[i]);
}

// ---------------------------------------------------------------------------
// factor installation
// ---------------------------------------------------------------------------
template <typename F>
__global__ void k_fill_slots(long long nslots, const int *__restrict__ src,
                             const double *__restrict__ lval, F *__restrict__ out) {
    for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < nslots;
         s += (long long)gridDim.x * blockDim.x) {
        const int k = src[s];
        out[s] = (k >= 0) ? static_cast<F>(lval[k]) : F(0);
    }
}

template <typename F>
__global__ void k_fill_inv(int n, const int *__restrict__ dpos, const double *__restrict__ lval,
                           F *__restrict__ inv) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double d = lval[dpos[i]];
        inv[i] = static_cast<F>(1.0 / static_cast<double>(static_cast<F>(d)));
    }
}

// Lower triangle copy (diagonal included); upper positions become 0.
__global__ void k_take_lower(int n, const int *__restrict__ rowptr, const int *__restrict__ col,
                             const double *__restrict__ src, double *__restrict__ dst) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) dst[k] = (col[k] <= i) ? src[k] : 0.0;
}

__global__ void k_set_int(int *p, int v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// Smallest row whose pivot is not > 0 or not finite, or with a non-finite
// off-diagonal value (the learned factor's guard).
__global__ void k_check_factor(int n, const int *__restrict__ rowptr, const int *__restrict__ col,
                               const int *__restrict__ dpos, const double *__restrict__ lval,
                               int *bad) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        bool ok = true;
        const double d = lval[dpos[i]];
        if (!(d > 0.0) || !isfinite(d)) ok = false;
        for (int k = rowptr[i]; k < dpos[i]; ++k)
            if (!isfinite(lval[k])) ok = false;
        if (!ok) atomicMin(bad, i);
    }
}

// IC(0) of A' on the device (Section 3; the LL^T form with L_ii = sqrt of the
// pivot), over the forward sweep's schedule: one launch per color, one
// wavefront per task, its chunks in order, and inside a chunk the rows of one
// level at a time (a row's lower neighbours lie in earlier colors, earlier
// chunks of its task or lower levels of its chunk, exactly the forward
// substitution's dependencies).  One lane computes one row, in the serial
// order of operations: for each lower entry k ascending,
//   L_ik = (a_ik - sum_{j<k, j in pat(i) and pat(k)} L_ij L_kj) / L_kk
// with the sum taken by a merge in ascending j, then the pivot
// d = a_ii - sum_k L_ik^2 ascending and L_ii = sqrt(d).  Multiplications and
// subtractions are not fused, so every entry equals the serial FP64
// factorization's bit for bit.  A pivot that is not > 0 or not finite lowers
// *bad to its row (the first failing row in serial order is the smallest:
// rows before it do not depend on it).
__device__ void ic0_row(int i, const int *__restrict__ rowptr, const int *__restrict__ col,
                        const double *__restrict__ val, const int *__restrict__ dpos,
                        double *__restrict__ L, int *bad) {
#pragma clang fp contract(off)
    const int r0 = rowptr[i], di = dpos[i];
    for (int p = r0; p < di; ++p) {
        const int k = col[p];
        double s = val[p];
        int a = r0, b = rowptr[k];
        const int be = dpos[k];
        while (a < p && b < be) {
            const int ca = col[a], cb = col[b];
            if (ca < cb) {
                ++a;
            } else if (ca > cb) {
                ++b;
            } else {
                s -= L[a] * L[b];
                ++a;
                ++b;
            }
        }
        L[p] = s / L[be];
    }
    double d = val[di];
    for (int p = r0; p < di; ++p) d -= L[p] * L[p];
    if (!(d > 0.0) || !isfinite(d)) atomicMin(bad, i);
    L[di] = sqrt(d);
}

__global__ __launch_bounds__(64) void k_ic0(const TaskRec *__restrict__ tasks,
                                            const Chunk *__restrict__ chunks,
                                            const uint32_t *__restrict__ meta, int task_base,
                                            int ntasks_color, const int *__restrict__ rowptr,
                                            const int *__restrict__ col, const double *__restrict__ val,
                                            const int *__restrict__ dpos, double *__restrict__ L, int *bad) {
    const int local = xcd_remap(blockIdx.x, gridDim.x);
    if (local >= ntasks_color) return;
    const TaskRec tr = tasks[task_base + local];
    const int t = static_cast<int>(threadIdx.x);
    for (int q = tr.c0; q < tr.c1; ++q) {
        const Chunk ch = q == tr.c0 ? tr.first : chunks[q];
        const int nr = ch.shape & 0xffff;
        const int i = ch.row0 + t;
        const int lev = t < nr ? static_cast<int>(meta[i] >> kMetaLevelShift) : -1;
        for (int lv = 0; lv < ch.depth; ++lv) {
            if (lev == lv) ic0_row(i, rowptr, col, val, dpos, L, bad);
            // the next level's rows (and the next chunk) read these entries
            // from memory: this wavefront's stores complete first
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            __builtin_amdgcn_wave_barrier();
        }
    }
}

// ---------------------------------------------------------------------------
// substitution sweep over the tasks of one color
// ---------------------------------------------------------------------------
template <typename F>
struct SweepArgs {
    const TaskRec *tasks;
    const Chunk *chunks;
    const uint32_t *meta;
    const int *scol;
    const F *sval;
    const F *inv;      // 1 / L_ii
};

// SW_APPLY: plain sweep.  SW_CG_FWD: forward sweep that first applies the CG
// update of its own rows (r -= alpha q) and substitutes the new r, with
// part[task] = sum of r_i^2.  SW_DOT_BWD: backward sweep with
// part[task] = sum of rdot_i z_i.
enum SweepMode : int { SW_APPLY = 0, SW_CG_FWD = 1, SW_DOT_BWD = 2 };

// Tasks (wavefronts) per workgroup of a per-color sweep launch.
constexpr int kSweepWaves = 1;
// Hybrid sweeps run the small trailing colors, up to this many tasks in all,
// as one dataflow launch (measured on 128^3: 700 beats 100 and 2200).
constexpr int kFlowTailTasks = 700;

struct CgArgs {
    double *r;
    const double *q;
    const double *rdot;
    double *part;
    const DevScalars *sc;
};

// One chunk of a task: see k_sweep.
struct NoWait {
    __device__ int pre() const { return 0; }
    __device__ void operator()(int) const {}
};

// Plain accesses: the per-color launches, where every value a task reads was
// written by an earlier launch or by the same wavefront.
struct PlainMem {
    template <typename T>
    __device__ __forceinline__ T gather(const T *out, int j) const { return out[j]; }
    template <typename T>
    __device__ __forceinline__ void store(T *out, int i, T v, uint32_t) const { out[i] = v; }
};

// Raw buffer accesses with an explicit cache policy (gfx950 CPol bits: 1 = sc0,
// 2 = nt, 16 = sc1).  Loads with sc0|nt miss in the CU's L1 and are served by
// the XCD's L2, which holds every store of that XCD's waves once the storing
// wave's vmcnt has drained; sc0 alone is not enough (a stale L1 line can keep
// serving it).  sc1 loads are coherent across XCDs.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, long long bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, static_cast<int>(bytes),
                                             0x00020000);
}
template <int AUX>
__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, int j, double) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, j * 8, 0, AUX));
}
template <int AUX>
__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, int j, float) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, j * 4, 0, AUX));
}
template <int AUX>
__device__ __forceinline__ int buf_load_i32(__amdgpu_buffer_rsrc_t r, int j) {
    return static_cast<int>(__builtin_amdgcn_raw_buffer_load_b32(r, j * 4, 0, AUX));
}
constexpr int kCpolL2 = 3;     // sc0 | nt
constexpr int kCpolSc1 = 16;

// Accesses of the single-launch sweep.  A task whose dependencies all lie in
// its own region reads them from its XCD's L2 (sc0|nt); a task with a dependency
// in another region reads every before-chunk value coherently across XCDs
// (sc1).  Rows that such tasks read carry the export bit and are written
// through to memory (sc1 stores); on the task's last chunk that write-through
// is deferred until the task has signalled its own region.
struct FlowMem {
    __amdgpu_buffer_rsrc_t rs;
    bool remote;
    bool defer_export;
    template <typename T>
    __device__ __forceinline__ T gather(const T *, int j) const {
        return remote ? buf_load<kCpolSc1>(rs, j, T()) : buf_load<kCpolL2>(rs, j, T());
    }
    template <typename T>
    __device__ __forceinline__ void store(T *out, int i, T v, uint32_t m) const {
        if ((m & kMetaExport) && !defer_export)
            __hip_atomic_store(out + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
            out[i] = v;
    }
};

// Rows stored in slot k of a chunk (see Chunk): a byte of cnt for jagged
// chunks, every row for padded ones.
__device__ __forceinline__ int slot_rows(const Chunk &ch, int k, bool jagged, int nr) {
    return (jagged && k < kJaggedMaxWidth)
               ? static_cast<int>((ch.cnt[(k >> 2) & 1] >> (8 * (k & 3))) & 0xffu)
               : nr;
}
// v of lane src/4 of the wavefront
__device__ __forceinline__ double lane_pull(double v, int src) {
    const int2 p = __builtin_bit_cast(int2, v);
    return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_ds_bpermute(src, p.x),
                                                __builtin_amdgcn_ds_bpermute(src, p.y)));
}
__device__ __forceinline__ float lane_pull(float v, int src) {
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(src, __builtin_bit_cast(int, v)));
}

// What one lane holds for one row of a chunk between the load phase (the
// chunk's schedule: every load that does not depend on other rows' results
// or on the CG vectors) and the finish phase.  vv/cc first hold the entries
// of the row at sorted position t (jagged chunks); the finish phase pulls
// them across to the lanes of their rows.
template <typename F, int KMAX>
struct RowRegs {
    F vv[KMAX];
    int cc[KMAX];
    uint32_t m;
    F dinv;
};

// Load phase of a chunk: every independent load at once, so they overlap.
// The schedule is read with ordinary loads.  Non-temporal ones were measured
// slower on every matrix once the slots became jagged (kNN graph and 27-point
// stencil solves 11-12 % slower, 7-point 0.5 %), although they do help the
// SpMV's matrix stream.
template <typename F, int KMAX>
__device__ __forceinline__ void sweep_load(const Chunk &ch, const uint32_t *__restrict__ meta,
                                           const int *__restrict__ scol, const F *__restrict__ sval,
                                           const F *__restrict__ inv, RowRegs<F, KMAX> &R) {
    const int t = static_cast<int>(threadIdx.x) & (kChunkRows - 1);
    const int nr = ch.shape & 0xffff, W = ch.shape >> 16;
    const bool jagged = W <= kJaggedMaxWidth;
    const int i = ch.row0 + t;
    R.m = 0;
    R.dinv = F(0);
    if (t < nr) {
        int sk = ch.off + t;
#pragma unroll
        for (int k = 0; k < KMAX; ++k)
            if (k < W) {
                const int rows_k = slot_rows(ch, k, jagged, nr);
                R.vv[k] = F(0);
                R.cc[k] = -1;
                if (t < rows_k) {
                    R.vv[k] = sval[sk];
                    R.cc[k] = scol[sk];
                }
                sk += rows_k;
            }
        R.m = meta[i];
        R.dinv = inv[i];
    }
}

// Finish phase of a chunk: the row's right-hand side (for the forward CG
// sweep r -= alpha q first), the pull of the jagged slots to their rows, the
// gathers of values final before the chunk (after `wait` has seen their
// producers), the in-chunk levels through LDS, and the store.
template <typename F, bool FWD, int KMAX, int MODE, typename TIn, typename TOut, class Wait,
          class Mem>
__device__ __forceinline__ void sweep_finish(const Chunk &ch, RowRegs<F, KMAX> &R,
                                             const int *__restrict__ scol,
                                             const F *__restrict__ sval,
                                             const TIn *__restrict__ in, TOut *__restrict__ out,
                                             const CgArgs &cg, double alpha, F *ys, double &dacc,
                                             const Wait &wait, int pre, const Mem &mem, F &y_out,
                                             uint32_t &m_out) {
    const int t = static_cast<int>(threadIdx.x) & (kChunkRows - 1);
    const int nr = ch.shape & 0xffff, W = ch.shape >> 16;
    const bool jagged = W <= kJaggedMaxWidth;
    const bool active = t < nr;
    const int i = ch.row0 + t;
    const int base = ch.off + t;
    const uint32_t m = R.m;
    F s = F(0);
    double rd = 0.0;
    if (active) {
        if (MODE == SW_CG_FWD) {
            const double ri = cg.r[i] - alpha * cg.q[i];
            cg.r[i] = ri;
            dacc += ri * ri;
            s = static_cast<F>(ri);
        } else {
            s = static_cast<F>(in[i]);
        }
        if (MODE == SW_DOT_BWD) rd = cg.rdot[i];
    }
    if (active && jagged) {
        // every row takes its entries from the lane of its sorted position
        const int src = static_cast<int>((m >> kMetaPosShift) & 63u) * 4;
#pragma unroll
        for (int k = 0; k < KMAX; ++k)
            if (k < W) {
                R.vv[k] = lane_pull(R.vv[k], src);
                R.cc[k] = __builtin_amdgcn_ds_bpermute(src, R.cc[k]);
            }
    }
    // values of other tasks are read only after their producers published them
    wait(pre);
    const int ne = m & kMetaNextMask, ni = (m >> kMetaInnerShift) & 63u, lev = m >> kMetaLevelShift;
    if (active) {
        // all gathers at once (the chunk width is uniform); slots that are not
        // before-chunk terms read a harmless valid address and are discarded
        F g[KMAX];
#pragma unroll
        for (int k = 0; k < KMAX; ++k)
            if (k < W) g[k] = static_cast<F>(mem.gather(out, R.cc[k] < 0 ? 0 : R.cc[k]));
#pragma unroll
        for (int k = 0; k < KMAX; ++k)
            if (k < W) s = (k < ne) ? s - R.vv[k] * g[k] : s;
        for (int k = KMAX; k < ne; ++k) {
            const int sl = base + k * nr;
            s -= sval[sl] * static_cast<F>(mem.gather(out, scol[sl]));
        }
    }
    for (int L = 0; L < ch.depth; ++L) {
        if (active && lev == L) {
#pragma unroll
            for (int k = 0; k < KMAX; ++k)
                if (k >= ne && k < ne + ni) s -= R.vv[k] * ys[R.cc[k] - ch.row0];
            for (int k = max(KMAX, ne); k < ne + ni; ++k) {
                const int sl = base + k * nr;
                s -= sval[sl] * ys[scol[sl] - ch.row0];
            }
            ys[t] = s * R.dinv;
        }
        // ys is this wavefront's own; its LDS operations execute in order,
        // so the next level's reads see this level's writes (the fences keep
        // the compiler from reordering them)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    F yv = F(0);
    if (active) {
        yv = ys[t];
        mem.store(out, i, static_cast<TOut>(yv), m);
        if (MODE == SW_DOT_BWD) dacc += rd * static_cast<double>(yv);
    }
    y_out = yv;
    m_out = m;
}

// One chunk of a task, both phases in a row.
template <typename F, bool FWD, int KMAX, int MODE, typename TIn, typename TOut, class Wait = NoWait,
          class Mem = PlainMem>
__device__ __forceinline__ void sweep_chunk(const Chunk &ch, const uint32_t *__restrict__ meta,
                                            const int *__restrict__ scol,
                                            const F *__restrict__ sval,
                                            const F *__restrict__ inv,
                                            const TIn *__restrict__ in, TOut *__restrict__ out,
                                            const CgArgs &cg, double alpha, F *ys, double &dacc,
                                            const Wait &wait, const Mem &mem, F &y_out,
                                            uint32_t &m_out) {
    // the first dependency a lane waits for, ahead of the chunk's loads
    const int pre = wait.pre();
    RowRegs<F, KMAX> R;
    sweep_load<F, KMAX>(ch, meta, scol, sval, inv, R);
    sweep_finish<F, FWD, KMAX, MODE, TIn, TOut>(ch, R, scol, sval, in, out, cg, alpha, ys, dacc, wait, pre,
                                                mem, y_out, m_out);
}

// One wavefront task: its chunks in the sweep's order (see k_sweep), and the
// task's partial sum in *part_out.
template <typename F, bool FWD, int KMAX, int MODE, typename TIn, typename TOut>
__device__ __forceinline__ void sweep_task(const TaskRec &tr, const Chunk *__restrict__ chunks,
                                           const uint32_t *__restrict__ meta,
                                           const int *__restrict__ scol, const F *__restrict__ sval,
                                           const F *__restrict__ inv, const TIn *__restrict__ in,
                                           TOut *__restrict__ out, const CgArgs &cg, F *ys,
                                           double *part_out) {
    const double alpha = (MODE == SW_CG_FWD) ? cg.sc->alpha : 0.0;
    double dacc = 0.0;
    F yv;
    uint32_t m;
    sweep_chunk<F, FWD, KMAX, MODE, TIn, TOut>(tr.first, meta, scol, sval, inv, in, out, cg, alpha,
                                               ys, dacc, NoWait(), PlainMem(), yv, m);
    const int nchunks = tr.c1 - tr.c0;
    for (int q = 1; q < nchunks; ++q) {
        // later chunks of this task read earlier chunks' results from memory:
        // this wavefront's stores complete before its next loads
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        const Chunk ch = chunks[FWD ? tr.c0 + q : tr.c1 - 1 - q];
        sweep_chunk<F, FWD, KMAX, MODE, TIn, TOut>(ch, meta, scol, sval, inv, in, out, cg, alpha,
                                                   ys, dacc, NoWait(), PlainMem(), yv, m);
    }
    if (MODE != SW_APPLY) {
        const double tsum = wave_sum(dacc);
        if ((threadIdx.x & 63) == 0) *part_out = tsum;
    }
}

// FWD: y_i = (r_i - sum_{j<i} L_ij y_j) / L_ii over the rows of one color.
// !FWD: z_i = (y_i - sum_{j>i} L_ji z_j) / L_ii.
// One wavefront per task, one lane per row of the current chunk.  All of the
// chunk's slots (up to KMAX per row in registers) are loaded at once, then all
// gathers of values final before the chunk, then the in-chunk terms level by
// level through LDS.  The per-row subtraction order is: before-chunk terms in
// ascending column order, then in-chunk terms in ascending column order.
// The arguments a wavefront needs first lead the list: the library is built
// with kernel-argument preloading, which puts the leading 56 bytes of a
// launch's arguments in scalar registers when the wavefront starts, so the
// task record and the stopping flag are loaded without waiting for them.
template <typename F, bool FWD, int KMAX, int MODE, typename TIn, typename TOut>
__global__ __launch_bounds__(64 * kSweepWaves) void k_sweep(const TaskRec *__restrict__ tasks,
                                                            const DevScalars *sc,
                                                            const uint32_t *__restrict__ meta,
                                                            const int *__restrict__ scol,
                                                            const F *__restrict__ sval,
                                                            const F *__restrict__ inv, int task_base,
                                                            int ntasks_color,
                                                            const Chunk *__restrict__ chunks,
                                                            int *bump, const TIn *__restrict__ in,
                                                            TOut *__restrict__ out, CgArgs cg) {
    __shared__ F ys_all[kSweepWaves][kChunkRows];
    // kSweepWaves independent tasks per workgroup, one per wavefront (fewer
    // workgroups to dispatch); consecutive tasks, so the XCD regions hold
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / 64);
    const int nwg = (ntasks_color + kSweepWaves - 1) / kSweepWaves;
    const int local = xcd_remap(blockIdx.x, nwg) * kSweepWaves + wave;
    // the task record and the stopping flag are read together (a surplus
    // wavefront of the last workgroup reads the color's last record), so
    // the launch waits for one memory round trip before its schedule loads
    const int task = task_base + min(local, ntasks_color - 1);
    const TaskRec tr = tasks[task];
    const bool running = *done_flag(sc) == DONE_RUNNING;   // sc is cg.sc
    // one test of both (bitwise, so neither load waits for the other);
    // wide tasks are run by k_sweep_wide
    if (running & (local < ntasks_color) & (tr.wide < 0))
        sweep_task<F, FWD, KMAX, MODE, TIn, TOut>(tr, chunks, meta, scol, sval, inv, in, out, cg,
                                                  ys_all[wave], cg.part ? cg.part + task : nullptr);
    // bumps the epoch of a dataflow launch that follows in the stream
    if (running && bump && blockIdx.x == 0 && threadIdx.x == 0) *bump += 1;
}

// Block of right-hand sides (columns ld apart): workgroup g runs task g of
// the color once per column, one wavefront per column (up to kColWaves
// columns per workgroup, blockIdx.y counts groups of them), so the schedule
// comes from HBM once and from the compute unit's caches for the other
// columns; every column computes exactly what k_sweep computes for it.
// Blocks of more than 64 rows run as chunk sequences (no wide tasks).
// Partial sums at part[c * part_ld + task]; columns whose solve has stopped
// skip their work.
template <typename F, bool FWD, int KMAX, int MODE, typename TIn, typename TOut>
__global__ __launch_bounds__(64 * kColWaves) void k_sweep_cols(const TaskRec *__restrict__ tasks,
                                                     const Chunk *__restrict__ chunks,
                                                     const uint32_t *__restrict__ meta,
                                                     const int *__restrict__ scol,
                                                     const F *__restrict__ sval,
                                                     const F *__restrict__ inv, int task_base,
                                                     int ntasks_color, const TIn *__restrict__ in,
                                                     TOut *__restrict__ out, CgArgs cg, int ld,
                                                     int part_ld, int ncols) {
    const int w = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    const int c = static_cast<int>(blockIdx.y) * kColWaves + w;
    if (c >= ncols) return;
    if (cg.sc && cg.sc[c].done != DONE_RUNNING) return;
    __shared__ F ys_all[kColWaves][kChunkRows];
    const int local = xcd_remap(blockIdx.x, gridDim.x);
    if (local >= ntasks_color) return;
    const int task = task_base + local;
    const TaskRec tr = tasks[task];
    const size_t off = static_cast<size_t>(c) * ld;
    CgArgs cc = cg;
    if (cc.r) cc.r += off;
    if (cc.q) cc.q += off;
    if (cc.rdot) cc.rdot += off;
    if (cc.sc) cc.sc += c;
    sweep_task<F, FWD, KMAX, MODE, TIn, TOut>(tr, chunks, meta, scol, sval, inv, in ? in + off : nullptr,
                                              out + off, cc, ys_all[w],
                                              cg.part ? cg.part + static_cast<size_t>(c) * part_ld + task
                                                      : nullptr);
}

// The turn of a CG iteration: the forward and then the backward substitution
// of the last color's tasks in one launch.  Blocks of one color are not
// coupled and no row lies in a later color, so the backward half of a task
// reads only values its own wavefront has just written; both halves are
// k_sweep's work for the task (the forward and backward schedules pack the
// color's blocks into the same tasks), so the results are bit-identical to
// two launches.
template <typename F, int KMAX>
__global__ __launch_bounds__(64) void k_sweep_turn(SweepArgs<F> fa, SweepArgs<F> ba, int task_base,
                                                   int ntasks, F *__restrict__ y, double *__restrict__ z,
                                                   CgArgs f, CgArgs g) {
    __shared__ F ys[kChunkRows];
    const int local = xcd_remap(blockIdx.x, ntasks);   // the grid has ntasks workgroups
    // task record and stopping flag read together, tested at once (as in
    // k_sweep; the turn's color has no wide task)
    const int task = task_base + min(local, ntasks - 1);
    const TaskRec tf = fa.tasks[task];
    if ((f.sc->done != DONE_RUNNING) | (local >= ntasks) | (tf.wide >= 0)) return;
    sweep_task<F, true, KMAX, SW_CG_FWD, double, F>(tf, fa.chunks, fa.meta, fa.scol, fa.sval, fa.inv, nullptr,
                                                     y, f, ys, f.part + task);
    // the backward half reads this wavefront's stores: they complete first
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    const TaskRec tb = ba.tasks[task];
    sweep_task<F, false, KMAX, SW_DOT_BWD, F, double>(tb, ba.chunks, ba.meta, ba.scol, ba.sval, ba.inv, y, z,
                                                       g, ys, g.part + task);
}

// Wide task (see WidePlan): one block of more than 64 rows, run piece by
// piece by a workgroup of WAVES wavefronts.  Wavefront w takes
// sub-chunk w of the piece, one lane per row.  Terms from outside the piece
// are gathered first (earlier pieces of the block were stored by this
// workgroup before the barrier that ends them); then the piece's levels run
// with a workgroup barrier after each, the values passing through LDS.
template <typename F, bool FWD, int KMAX, int MODE, typename TIn, typename TOut, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_sweep_wide(
    const int *__restrict__ wtask, const int *__restrict__ piece_ptr,
    const WidePiece *__restrict__ pieces, const Chunk *__restrict__ subs,
    const uint32_t *__restrict__ wmeta, const int *__restrict__ wlev, const int *__restrict__ scol,
    const F *__restrict__ sval, const F *__restrict__ inv, int w_base, const TIn *__restrict__ in,
    TOut *__restrict__ out, CgArgs cg) {
    if (cg.sc && cg.sc->done != DONE_RUNNING) return;
    __shared__ F ys[64 * WAVES];
    const int t = static_cast<int>(threadIdx.x) & 63;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    const int w = w_base + static_cast<int>(blockIdx.x);
    const double alpha = (MODE == SW_CG_FWD) ? cg.sc->alpha : 0.0;
    double dacc = 0.0;
    for (int pc = piece_ptr[w]; pc < piece_ptr[w + 1]; ++pc) {
        const WidePiece P = pieces[pc];
        int row0 = 0, off = 0, nr = 0, W = 0;
        if (wave < P.nsub) {
            const Chunk sc = subs[P.sub0 + wave];
            row0 = sc.row0;
            off = sc.off;
            nr = sc.shape & 0xffff;
            W = sc.shape >> 16;
        }
        const bool active = t < nr;
        const int i = row0 + t;
        const int base = off + t;
        F vv[KMAX];
        int cc[KMAX];
        uint32_t m = 0;
        int lev = 0;
        F s = F(0), dinv = F(0);
        double rd = 0.0;
        if (active) {
#pragma unroll
            for (int k = 0; k < KMAX; ++k)
                if (k < W) {
                    vv[k] = sval[base + k * nr];
                    cc[k] = scol[base + k * nr];
                }
            m = wmeta[i];
            lev = wlev[i];
            dinv = inv[i];
            if (MODE == SW_CG_FWD) {
                const double ri = cg.r[i] - alpha * cg.q[i];
                cg.r[i] = ri;
                dacc += ri * ri;
                s = static_cast<F>(ri);
            } else {
                s = static_cast<F>(in[i]);
            }
            if (MODE == SW_DOT_BWD) rd = cg.rdot[i];
        }
        const int ne = static_cast<int>(m & 0xffffu), ni = static_cast<int>(m >> 16);
        if (active) {
            // terms from outside the piece, ascending; the padding and the
            // piece's own slots read a harmless valid address
            F g[KMAX];
#pragma unroll
            for (int k = 0; k < KMAX; ++k)
                if (k < W) g[k] = static_cast<F>(out[cc[k] < 0 ? 0 : cc[k]]);
#pragma unroll
            for (int k = 0; k < KMAX; ++k)
                if (k < W) s = (k < ne) ? s - vv[k] * g[k] : s;
            for (int k = KMAX; k < ne; ++k) {
                const int sl = base + k * nr;
                s -= sval[sl] * static_cast<F>(out[scol[sl]]);
            }
        }
        for (int L = 0; L < P.depth; ++L) {
            if (active && lev == L) {
#pragma unroll
                for (int k = 0; k < KMAX; ++k)
                    if (k >= ne && k < ne + ni) s -= vv[k] * ys[cc[k] - P.row0];
                for (int k = max(KMAX, ne); k < ne + ni; ++k) {
                    const int sl = base + k * nr;
                    s -= sval[sl] * ys[scol[sl] - P.row0];
                }
                ys[i - P.row0] = s * dinv;
            }
            __syncthreads();
        }
        if (active) {
            const F yv = ys[i - P.row0];
            out[i] = static_cast<TOut>(yv);
            if (MODE == SW_DOT_BWD) dacc += rd * static_cast<double>(yv);
        }
        // the next piece gathers these values from memory
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        __syncthreads();
    }
    if (MODE != SW_APPLY) {
        const double tsum = block_sum<64 * WAVES>(dacc);
        if (threadIdx.x == 0) cg.part[wtask[w]] = tsum;
    }
}

// Dataflow sweep: the tasks of every color (or of a run of colors) in one
// launch.  The launch table lists the tasks in processing order (forward:
// colors ascending, backward: descending), and every task a task waits for
// sits at a smaller table position; how positions map to workgroups and why
// that guarantees progress is described at k_sweep_flow.
//
// Workgroups are dealt to the XCDs round robin, so the workgroups with one
// value of b mod 8 (one region of the domain in every color) share an XCD
// and its L2.  A finished task raises two flags holding (epoch << 4 | XCC id):
//   flag_loc, after its stores have reached L2 (read by same-region tasks
//             through L2), and
//   flag_rem, after its exported rows have been written through to memory
//             (read coherently by tasks that have a dependency elsewhere).
// A same-region waiter checks that the producer ran on its own XCD; if the
// round-robin placement ever failed, the sweep reports an error instead of
// reading a value that might not be visible.  The epoch is bumped before
// every launch (by a one-thread kernel, or in the hybrid mode by a kernel that
// runs anyway), so flags are never reset between sweeps.  A wait that exceeds
// the spin limit sets *err and continues, so every wavefront always exits.
struct FlowArgs {
    const int *epoch;
    int *flag_loc;
    int *flag_rem;
    const int *deps;
    const int *wg_task;
    int ntasks;
    int pos0, pos1;      // table positions this launch runs
    int dep_done_below;  // dependencies with a smaller task id are already final
    int *bump;           // if set, block 0 bumps this (the other sweep's) epoch
    int spin_limit;
    int *err;            // 1: spin limit, 2: placement
};

__global__ void k_bump_epoch(int *epoch, const DevScalars *sc) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && !(sc && sc->done != DONE_RUNNING)) *epoch += 1;
}

__device__ __forceinline__ int xcc_id() {
    int v;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
    return v & 15;
}

struct FlowWait {
    const FlowArgs *fa;
    __amdgpu_buffer_rsrc_t rs_loc;
    int task, epoch, xcc;
    int d0, nd;
    bool remote;
    __device__ int pre() const {
        const int l = static_cast<int>(threadIdx.x);
        return l < nd ? fa->deps[d0 + l] : 0;
    }
    // one lane per dependency polls its flag
    __device__ void operator()(int first) const {
        for (int l = static_cast<int>(threadIdx.x); l < nd; l += 64) {
            const int dep = l < 64 ? first : fa->deps[d0 + l];
            if (dep < fa->dep_done_below) continue;   // written by an earlier launch
            int spins = 0;
            while (true) {
                const int v = remote ? __hip_atomic_load(fa->flag_rem + dep, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT)
                                     : buf_load_i32<kCpolL2>(rs_loc, dep);
                if ((v >> 4) >= epoch) {
                    if (!remote && (v & 15) != xcc)
                        __hip_atomic_store(fa->err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                ++spins;
                // after any failure every other wait gives up at once
                if ((spins & 255) == 0 &&
                    __hip_atomic_load(fa->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                    break;
                if (spins > fa->spin_limit) {
                    __hip_atomic_store(fa->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
        }
        // the wavefront's lanes reconverge here; the gathers that follow are
        // issued after every flag was seen
    }
};

// Persistent form: the grid holds R resident workgroups (R a multiple of 8,
// or R = ntasks) and workgroup g runs the table positions g, g + R, g + 2R, ...
// in order, all in one region.  Dependencies always sit at smaller positions,
// so the smallest unfinished position is always being worked on: with every
// workgroup resident, the sweep completes.
template <typename F, bool FWD, int KMAX, int MODE, typename TIn, typename TOut>
__global__ __launch_bounds__(64) void k_sweep_flow(const TaskRec *__restrict__ tasks,
                                                   const Chunk *__restrict__ chunks,
                                                   const uint32_t *__restrict__ meta,
                                                   const int *__restrict__ scol,
                                                   const F *__restrict__ sval,
                                                   const F *__restrict__ inv, FlowArgs fa, int n,
                                                   const TIn *__restrict__ in,
                                                   TOut *__restrict__ out, CgArgs cg) {
    if (cg.sc && cg.sc->done != DONE_RUNNING) return;
    if (fa.bump && blockIdx.x == 0 && threadIdx.x == 0) *fa.bump += 1;
    __shared__ F ys[kChunkRows];
    const int epoch = *fa.epoch;
    const int xcc = xcc_id();
    const double alpha = (MODE == SW_CG_FWD) ? cg.sc->alpha : 0.0;
    const int word = (epoch << 4) | xcc;
    const __amdgpu_buffer_rsrc_t rs_out = make_rsrc(out, static_cast<long long>(n) * sizeof(TOut));
    const __amdgpu_buffer_rsrc_t rs_loc = make_rsrc(fa.flag_loc, 4LL * fa.ntasks);
    for (int pos = fa.pos0 + static_cast<int>(blockIdx.x); pos < fa.pos1; pos += gridDim.x) {
        const int task = fa.wg_task[pos];
        const TaskRec tr = tasks[task];
        const int kind = tr.kind_ndeps & 3, nchunks = tr.c1 - tr.c0;
        const bool remote = (kind & kTaskRemote) != 0;
        double dacc = 0.0;
        const FlowWait wait{&fa, rs_loc, task, epoch, xcc, tr.dep0, tr.kind_ndeps >> 2, remote};
        F yv;
        uint32_t m;
        sweep_chunk<F, FWD, KMAX, MODE, TIn, TOut>(tr.first, meta, scol, sval, inv, in, out, cg,
                                                   alpha, ys, dacc, wait,
                                                   FlowMem{rs_out, remote, nchunks == 1}, yv, m);
        for (int q = 1; q < nchunks; ++q) {
            __builtin_amdgcn_s_waitcnt(0);   // this chunk's stores are complete before they are read
            __syncthreads();
            const Chunk ch = chunks[FWD ? tr.c0 + q : tr.c1 - 1 - q];
            sweep_chunk<F, FWD, KMAX, MODE, TIn, TOut>(ch, meta, scol, sval, inv, in, out, cg, alpha,
                                                       ys, dacc, NoWait(),
                                                       FlowMem{rs_out, remote, q == nchunks - 1}, yv, m);
        }
        if (MODE != SW_APPLY) {
            const double tsum = wave_sum(dacc);
            if (threadIdx.x == 0) cg.part[task] = tsum;
        }
        // signal the region: every store of this wavefront has reached L2
        __builtin_amdgcn_s_waitcnt(0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (threadIdx.x == 0)
            __hip_atomic_store(fa.flag_loc + task, word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (kind & kTaskExports) {
            // then write the last chunk's exported rows through and signal the
            // other regions
            const Chunk last = nchunks == 1 ? tr.first : chunks[FWD ? tr.c1 - 1 : tr.c0];
            const int nr = last.shape & 0xffff;
            if (static_cast<int>(threadIdx.x) < nr && (m & kMetaExport))
                __hip_atomic_store(out + last.row0 + threadIdx.x, static_cast<TOut>(yv),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_s_waitcnt(0);
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            if (threadIdx.x == 0)
                __hip_atomic_store(fa.flag_rem + task, word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// static scratch of the allocation-free entry point (iccg_spmv_dot_noalloc)
// ---------------------------------------------------------------------------
// The SpMV's per-workgroup partial sums, one double per workgroup: 2^18 of
// them cover n <= 2^24 rows (a workgroup covers 64 rows of a matrix with
// rows wider than 8 entries, 128 otherwise).  Each GPU holds its own copy
// for the life of the process; host code reaches it only through the
// address hipGetSymbolAddress returns for the current device (resolved in
// iccg_setup), never through the array's name.
constexpr int kNoAllocMaxRows = 1 << 24;
constexpr int kNoAllocParts = 1 << 18;
__device__ __align__(256) double scratch[kNoAllocParts];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev (the current device), resolved
// once per device.
int resolve_scratch(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return set_error(ICCG_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return ICCG_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return set_error(ICCG_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double *>(ptr);
    return ICCG_OK;
}

double *scratch_for(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[dev];
}

int grid_for(long long items, int threads, int cap) {
    long long g = (items + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return static_cast<int>(g);
}

// part: one partial sum per workgroup (c->spmv_blocks of them); NULL = the
// context's partial buffer
int launch_spmv(iccg_ctx *c, int mode, const double *x, double *y, const double *b,
                const DevScalars *sc, double *part = nullptr) {
    dim3 grid(c->spmv_blocks), block(64);
    if (!part) part = c->part.p;
    if (c->prof) c->prof->begin(c->work);
#define SPMV_ARGS c->n, c->nslices, c->sell_rec.p, sc, c->sell_col.p, c->sell_val.p, x, y, b, part
#define SPMV_W(M)                                                                              \
    switch (c->sell_wmax) {                                                                    \
        case 8: hipLaunchKernelGGL((k_spmv<M, 8>), grid, block, 0, c->work, SPMV_ARGS); break;   \
        case 16: hipLaunchKernelGGL((k_spmv<M, 16>), grid, block, 0, c->work, SPMV_ARGS); break; \
        default: hipLaunchKernelGGL((k_spmv<M, 32>), grid, block, 0, c->work, SPMV_ARGS); break; \
    }
    if (mode == SP_PLAIN) {
        SPMV_W(SP_PLAIN)
    } else {
        SPMV_W(SP_RESID)
    }
#undef SPMV_W
#undef SPMV_ARGS
    if (c->prof) c->prof->end(c->work, PK_SPMV);
    HIP_CHECK(hipGetLastError());
    return ICCG_OK;
}

template <typename F>
SweepArgs<F> sweep_args(const iccg_ctx *c, const DevSweep &s) {
    SweepArgs<F> a;
    a.tasks = s.tasks.p;
    a.chunks = s.chunks.p;
    a.meta = s.meta.p;
    a.scol = s.scol.p;
    if constexpr (sizeof(F) == 4) {
        a.sval = s.sval32.p;
        a.inv = c->inv32.p;
    } else {
        a.sval = s.sval64.p;
        a.inv = c->inv64.p;
    }
    return a;
}

// Workgroups of a persistent single-launch sweep.  Every workgroup must be
// resident at once, so the count is bounded by the occupancy the kernel's own
// register and LDS use allow (the runtime's occupancy query can report more
// 64-thread workgroups per CU than fit), and by default by 8 per CU, the
// fastest measured setting.  A multiple of 8, so a workgroup's table
// positions all fall in one region; at most one per task.  Cached per kernel.
int resident_grid(iccg_ctx *c, const void *kfn, int ntasks, int *grid) {
    auto it = c->resident.find(kfn);
    int per_cu = 0;
    if (it != c->resident.end()) {
        per_cu = it->second;
    } else {
        HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, 64, 0));
        hipFuncAttributes fa;
        HIP_CHECK(hipFuncGetAttributes(&fa, kfn));
        // one wave per workgroup: 4 SIMDs x min(8, 512 / VGPRs rounded up to 8)
        const int vgprs = std::max(8, (fa.numRegs + 7) / 8 * 8);
        per_cu = std::min(per_cu, 4 * std::min(8, 512 / vgprs));
        if (fa.sharedSizeBytes > 0)
            per_cu = std::min<int>(per_cu, static_cast<int>((160 * 1024) / fa.sharedSizeBytes));
        c->resident[kfn] = per_cu;
    }
    long long r = static_cast<long long>(std::min(per_cu, 8)) * c->num_cu;
    if (c->opt.sweep_grid > 0)
        r = std::min<long long>(static_cast<long long>(per_cu) * c->num_cu, std::max(c->opt.sweep_grid, 8));
    r -= r % 8;
    if (r < 8) return set_error(ICCG_EHIP, "single-launch sweep: no resident capacity for its kernel");
    *grid = static_cast<int>(std::min<long long>(r, std::max(ntasks, 1)));
    return ICCG_OK;
}

// One dataflow launch over the table positions [pos0, pos1) of a sweep.
template <typename F, bool FWD, int MODE, typename TIn, typename TOut>
int launch_flow(iccg_ctx *c, DevSweep &d, const SweepArgs<F> &a, int pos0, int pos1,
                int dep_done_below, int *bump, const TIn *pin, TOut *pout, const CgArgs &cg) {
    FlowArgs fa;
    fa.epoch = d.epoch.p;
    fa.flag_loc = d.flag_loc.p;
    fa.flag_rem = d.flag_rem.p;
    fa.deps = d.deps.p;
    fa.wg_task = d.wg_task.p;
    fa.ntasks = d.ntasks;
    fa.pos0 = pos0;
    fa.pos1 = pos1;
    fa.dep_done_below = dep_done_below;
    fa.bump = bump;
    fa.spin_limit = 1 << 18;
    fa.err = c->sweep_err.p;
    const void *kfn = nullptr;
    switch (d.kmax) {
        case 4: kfn = reinterpret_cast<const void *>(&k_sweep_flow<F, FWD, 4, MODE, TIn, TOut>); break;
        case 6:
        case 8: kfn = reinterpret_cast<const void *>(&k_sweep_flow<F, FWD, 8, MODE, TIn, TOut>); break;
        case 16: kfn = reinterpret_cast<const void *>(&k_sweep_flow<F, FWD, 16, MODE, TIn, TOut>); break;
        default: kfn = reinterpret_cast<const void *>(&k_sweep_flow<F, FWD, 32, MODE, TIn, TOut>); break;
    }
    int R = 0;
    ICCG_CHECK(resident_grid(c, kfn, pos1 - pos0, &R));
    c->last_resident = R;
    const dim3 grid(R), block(64);
#define FLOW_ARGS a.tasks, a.chunks, a.meta, a.scol, a.sval, a.inv, fa, c->n, pin, pout, cg
    switch (d.kmax) {
        case 4: hipLaunchKernelGGL((k_sweep_flow<F, FWD, 4, MODE, TIn, TOut>), grid, block, 0, c->work, FLOW_ARGS); break;
        case 6:
        case 8: hipLaunchKernelGGL((k_sweep_flow<F, FWD, 8, MODE, TIn, TOut>), grid, block, 0, c->work, FLOW_ARGS); break;
        case 16: hipLaunchKernelGGL((k_sweep_flow<F, FWD, 16, MODE, TIn, TOut>), grid, block, 0, c->work, FLOW_ARGS); break;
        default: hipLaunchKernelGGL((k_sweep_flow<F, FWD, 32, MODE, TIn, TOut>), grid, block, 0, c->work, FLOW_ARGS); break;
    }
#undef FLOW_ARGS
    HIP_CHECK(hipGetLastError());
    return ICCG_OK;
}

// All colors of one sweep direction (colors ascending for the forward sweep,
// descending for the backward sweep):
//   per-color: one launch per color;
//   single:    one dataflow launch for all of them;
//   hybrid:    one launch per large color, and the small colors (the last
//              ones of the forward sweep, the first ones of the backward
//              sweep) in one dataflow launch.  The first forward launch bumps
//              the forward epoch, the forward dataflow launch the backward
//              one, so no launch is added (a backward sweep on its own gets
//              its bump from the entry point).
// turn: the last color is left to k_sweep_turn (per-color launches only).
template <typename F, bool FWD, int MODE>
int launch_sweep_t(iccg_ctx *c, const void *in, void *out, const CgArgs &cg, bool turn = false) {
    using TIn = typename std::conditional<FWD, double, F>::type;
    using TOut = typename std::conditional<FWD, F, double>::type;
    DevSweep &d = FWD ? c->fwd : c->bwd;
    const SweepArgs<F> a = sweep_args<F>(c, d);
    const TIn *pin = static_cast<const TIn *>(in);
    TOut *pout = static_cast<TOut *>(out);
    if (c->prof) c->prof->begin(c->work);
    if (c->opt.sweep_launch == 1) {
        hipLaunchKernelGGL(k_bump_epoch, dim3(1), dim3(64), 0, c->work, d.epoch.p, cg.sc);
        ICCG_CHECK((launch_flow<F, FWD, MODE>(c, d, a, 0, d.ntasks, 0, nullptr, pin, pout, cg)));
        if (c->prof) c->prof->end(c->work, FWD ? PK_FWD : PK_BWD);
        return ICCG_OK;
    }
    // colors [tail, ncolors) run as one dataflow launch in the hybrid mode
    const int tail = c->opt.sweep_launch == 2 ? c->flow_tail : c->ncolors;
    const int tail_tasks = d.color_task_ptr[c->ncolors] - d.color_task_ptr[tail];
#define SWEEP_ARGS a.tasks, cg.sc, a.meta, a.scol, a.sval, a.inv, t0, t1 - t0, a.chunks, bump, pin, pout, cg
    int launched = 0;
    // wide tasks (per-color launches only): values and LDS-level pieces of
    // the blocks of more than 64 rows
    const DevWide &dw = d.wide;
    const F *wsval = nullptr;
    if constexpr (sizeof(F) == 4) wsval = dw.sval32.p; else wsval = dw.sval64.p;
#define WIDE_ARGS dw.task.p, dw.piece_ptr.p, dw.pieces.p, dw.subs.p, dw.wmeta.p, dw.wlev.p, dw.scol.p, \
                  wsval, a.inv, w0, pin, pout, cg
    auto per_color = [&](int col, int *bump) -> int {
        const int t0 = d.color_task_ptr[col], t1 = d.color_task_ptr[col + 1];
        if (t1 == t0) return ICCG_OK;
        const int w0 = dw.nwide > 0 ? dw.color_ptr[col] : 0;
        const int nw = dw.nwide > 0 ? dw.color_ptr[col + 1] - w0 : 0;
        if (t1 - t0 > nw || bump) {
            ++launched;
            const dim3 grid((t1 - t0 + kSweepWaves - 1) / kSweepWaves), block(64 * kSweepWaves);
            switch (d.color_kmax[col]) {
                case 4: hipLaunchKernelGGL((k_sweep<F, FWD, 4, MODE, TIn, TOut>), grid, block, 0, c->work, SWEEP_ARGS); break;
                case 6: hipLaunchKernelGGL((k_sweep<F, FWD, 6, MODE, TIn, TOut>), grid, block, 0, c->work, SWEEP_ARGS); break;
                case 8: hipLaunchKernelGGL((k_sweep<F, FWD, 8, MODE, TIn, TOut>), grid, block, 0, c->work, SWEEP_ARGS); break;
                case 16: hipLaunchKernelGGL((k_sweep<F, FWD, 16, MODE, TIn, TOut>), grid, block, 0, c->work, SWEEP_ARGS); break;
                case 28: hipLaunchKernelGGL((k_sweep<F, FWD, 28, MODE, TIn, TOut>), grid, block, 0, c->work, SWEEP_ARGS); break;
                default: hipLaunchKernelGGL((k_sweep<F, FWD, 32, MODE, TIn, TOut>), grid, block, 0, c->work, SWEEP_ARGS); break;
            }
            HIP_CHECK(hipGetLastError());
        }
        if (nw > 0) {
            ++launched;
            // the piece size the plan was built with: 64 rows per wavefront,
            // wide_waves(max width) wavefronts
            const dim3 grid(nw), block(64 * wide_waves(d.max_width));
            switch (d.kmax) {
                case 4: hipLaunchKernelGGL((k_sweep_wide<F, FWD, 4, MODE, TIn, TOut, wide_waves(4)>), grid, block, 0, c->work, WIDE_ARGS); break;
                case 6:
                case 8: hipLaunchKernelGGL((k_sweep_wide<F, FWD, 8, MODE, TIn, TOut, wide_waves(8)>), grid, block, 0, c->work, WIDE_ARGS); break;
                case 16: hipLaunchKernelGGL((k_sweep_wide<F, FWD, 16, MODE, TIn, TOut, wide_waves(16)>), grid, block, 0, c->work, WIDE_ARGS); break;
                default: hipLaunchKernelGGL((k_sweep_wide<F, FWD, 32, MODE, TIn, TOut, wide_waves(32)>), grid, block, 0, c->work, WIDE_ARGS); break;
            }
            HIP_CHECK(hipGetLastError());
        }
        return ICCG_OK;
    };
    const int skip = (turn && tail_tasks == 0) ? 1 : 0;
    if (FWD) {
        for (int col = 0; col < tail - skip; ++col)
            ICCG_CHECK(per_color(col, col == 0 && tail_tasks > 0 ? d.epoch.p : nullptr));
        if (tail_tasks > 0) {
            if (tail == 0)
                hipLaunchKernelGGL(k_bump_epoch, dim3(1), dim3(64), 0, c->work, d.epoch.p, cg.sc);
            // positions of colors >= tail are the table's last tail_tasks
            ICCG_CHECK((launch_flow<F, FWD, MODE>(c, d, a, d.ntasks - tail_tasks, d.ntasks,
                                                   d.color_task_ptr[tail], c->bwd.epoch.p, pin, pout, cg)));
            ++launched;
        }
    } else {
        if (tail_tasks > 0) {
            // the backward sweep starts with the small colors: the table's
            // first tail_tasks positions, all of whose dependencies are inside
            ICCG_CHECK((launch_flow<F, FWD, MODE>(c, d, a, 0, tail_tasks, 0, nullptr, pin, pout, cg)));
            ++launched;
        }
        for (int col = tail - 1 - skip; col >= 0; --col) ICCG_CHECK(per_color(col, nullptr));
    }
#undef SWEEP_ARGS
#undef WIDE_ARGS
    if (c->prof) c->prof->end(c->work, FWD ? PK_FWD : PK_BWD, launched);
    return ICCG_OK;
}

// A failed single-launch sweep (error word set by a wavefront) is reported
// and the word is cleared, so the context stays usable (for instance with
// per-color launches).
int report_sweep_err(iccg_ctx *c, int err) {
    if (!err) return ICCG_OK;
    (void)hipMemsetAsync(c->sweep_err.p, 0, sizeof(int), c->work);
    (void)hipStreamSynchronize(c->work);
    if (err == 2)
        return set_error(ICCG_EHIP, "single-launch sweep: a producer task ran on another XCD than "
                                    "its region (round-robin placement failed); use per-color launches");
    return set_error(ICCG_EHIP, "single-launch sweep: a dependency wait exceeded its spin limit");
}

// fails loudly if a dependency wait of the single-launch sweep failed
int check_sweep_err(iccg_ctx *c) {
    if (c->opt.sweep_launch == 0) return ICCG_OK;
    int err = 0;
    HIP_CHECK(hipMemcpyAsync(&err, c->sweep_err.p, sizeof(int), hipMemcpyDeviceToHost, c->work));
    HIP_CHECK(hipStreamSynchronize(c->work));
    return report_sweep_err(c, err);
}

// The flag words hold (epoch << 4 | XCC id), so the epoch must stay below
// 2^27: before it could get there, flags and epochs are cleared (host path,
// never inside a captured graph).  `sweeps` bounds the launches to come.
int flow_guard(iccg_ctx *c, long long sweeps) {
    if (c->opt.sweep_launch == 0) return ICCG_OK;
    if (c->flow_sweeps + sweeps < (1LL << 26)) {
        c->flow_sweeps += sweeps;
        return ICCG_OK;
    }
    for (DevSweep *d : {&c->fwd, &c->bwd}) {
        const size_t nf = sizeof(int) * static_cast<size_t>(std::max(d->ntasks, 1));
        HIP_CHECK(hipMemsetAsync(d->flag_loc.p, 0, nf, c->work));
        HIP_CHECK(hipMemsetAsync(d->flag_rem.p, 0, nf, c->work));
        HIP_CHECK(hipMemsetAsync(d->epoch.p, 0, sizeof(int), c->work));
    }
    c->flow_sweeps = sweeps;
    return ICCG_OK;
}

template <bool FWD, int MODE>
int launch_sweep(iccg_ctx *c, const void *in, void *out, const CgArgs &cg, bool turn = false) {
    return c->fp32() ? launch_sweep_t<float, FWD, MODE>(c, in, out, cg, turn)
                     : launch_sweep_t<double, FWD, MODE>(c, in, out, cg, turn);
}

void *ytmp(iccg_ctx *c);

// The last color of the CG sweeps in one k_sweep_turn launch: per-color
// launches, no wide task in that color, the same task packing both ways, and
// not inside an instrumented solve (whose per-sweep times it would mix).
bool turn_ok(const iccg_ctx *c) {
    if (!c->opt.fuse_turn || c->opt.sweep_launch != 0 || c->prof || c->ncolors < 1) return false;
    if (c->fwd.color_task_ptr != c->bwd.color_task_ptr) return false;
    const int last = c->ncolors - 1;
    for (const DevSweep *d : {&c->fwd, &c->bwd}) {
        const DevWide &w = d->wide;
        if (w.nwide > 0 && w.color_ptr[last + 1] > w.color_ptr[last]) return false;
    }
    return true;
}

template <typename F>
int launch_turn_t(iccg_ctx *c, const CgArgs &f, const CgArgs &g) {
    const int last = c->ncolors - 1;
    const int t0 = c->fwd.color_task_ptr[last], nt = c->fwd.color_task_ptr[last + 1] - t0;
    if (nt <= 0) return ICCG_OK;
    const SweepArgs<F> fa = sweep_args<F>(c, c->fwd), ba = sweep_args<F>(c, c->bwd);
    F *y = static_cast<F *>(ytmp(c));
    const int K = std::max(c->fwd.color_kmax[last], c->bwd.color_kmax[last]);
    const dim3 grid(nt), block(64);
#define TURN_ARGS fa, ba, t0, nt, y, c->z.p, f, g
    switch (K) {
        case 4: hipLaunchKernelGGL((k_sweep_turn<F, 4>), grid, block, 0, c->work, TURN_ARGS); break;
        case 6: hipLaunchKernelGGL((k_sweep_turn<F, 6>), grid, block, 0, c->work, TURN_ARGS); break;
        case 8: hipLaunchKernelGGL((k_sweep_turn<F, 8>), grid, block, 0, c->work, TURN_ARGS); break;
        case 16: hipLaunchKernelGGL((k_sweep_turn<F, 16>), grid, block, 0, c->work, TURN_ARGS); break;
        case 28: hipLaunchKernelGGL((k_sweep_turn<F, 28>), grid, block, 0, c->work, TURN_ARGS); break;
        default: hipLaunchKernelGGL((k_sweep_turn<F, 32>), grid, block, 0, c->work, TURN_ARGS); break;
    }
#undef TURN_ARGS
    HIP_CHECK(hipGetLastError());
    return ICCG_OK;
}

CgArgs no_cg() {
    CgArgs a;
    std::memset(&a, 0, sizeof(a));
    return a;
}

void *ytmp(iccg_ctx *c) { return c->fp32() ? static_cast<void *>(c->y32.p) : c->y64.p; }

int launch_reduce(iccg_ctx *c, int np, int op, double *out) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kReduceThreads), 0, c->work, c->part.p, np,
                       c->scal.p, op, out, c->hist.p, 0, 0);
    HIP_CHECK(hipGetLastError());
    return ICCG_OK;
}

// One CG iteration (all kernels return at once after the stopping test passed):
//   1. x += alpha p (the previous iteration's step, deferred to here), then
//      p = z + beta p (alpha = beta = 0 and p = 0 before the first iteration)
//   2. SpMV:     q = A p, alpha = rho / (p, q)
//   3. forward:  r -= alpha q, ||r||^2 partials, y = L^{-1} r
//   4. backward: z = L^{-T} y, (r, z) partials
//   5. stopping test on ||r||, then beta = (r, z)/rho, rho = (r, z)
int enqueue_iteration(iccg_ctx *c, long long j) {
    (void)j;
    DevScalars *sc = c->scal.p;
    double *p = c->p.p;
    hipLaunchKernelGGL(k_update_p, dim3(c->nslices), dim3(64), 0, c->work, c->n, c->nslices,
                       c->sell_order.p, c->x.p, p, c->z.p, sc);
    HIP_CHECK(hipGetLastError());
    ICCG_CHECK(launch_spmv(c, SP_PLAIN, p, c->q.p, nullptr, sc));
    ICCG_CHECK(launch_reduce(c, c->spmv_blocks, OP_ALPHA, nullptr));
    CgArgs f = no_cg();
    f.r = c->r.p;
    f.q = c->q.p;
    f.part = c->part_rr.p;
    f.sc = sc;
    CgArgs g = no_cg();
    g.rdot = c->r.p;
    g.part = c->part.p;
    g.sc = sc;
    const bool turn = turn_ok(c);
    ICCG_CHECK((launch_sweep<true, SW_CG_FWD>(c, nullptr, ytmp(c), f, turn)));
    if (turn) ICCG_CHECK(c->fp32() ? launch_turn_t<float>(c, f, g) : launch_turn_t<double>(c, f, g));
    ICCG_CHECK((launch_sweep<false, SW_DOT_BWD>(c, ytmp(c), c->z.p, g, turn)));
    hipLaunchKernelGGL(k_reduce_rr_beta, dim3(1), dim3(kReduceThreads), 0, c->work, c->part_rr.p,
                       c->fwd.ntasks, c->part.p, c->bwd.ntasks, sc, c->hist.p, 0, 0);
    HIP_CHECK(hipGetLastError());
    return ICCG_OK;
}

// A batch of iterations; one captured graph serves every batch.
int enqueue_batch(iccg_ctx *c, long long j0, int iters) {
    for (int k = 0; k < iters; ++k) ICCG_CHECK(enqueue_iteration(c, j0 + k));
    return ICCG_OK;
}

int run_batch(iccg_ctx *c, long long j0, int iters) {
    if (!c->opt.use_graph) return enqueue_batch(c, j0, iters);
    if (!c->graph || c->graph_iters != iters) {
        if (c->graph) {
            HIP_CHECK(hipGraphExecDestroy(c->graph));
            c->graph = nullptr;
        }
        HIP_CHECK(hipStreamBeginCapture(c->work, hipStreamCaptureModeThreadLocal));
        int st = enqueue_batch(c, 1, iters);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c->work, &g);
        if (st != ICCG_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return set_error(ICCG_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            c->graph = nullptr;
            return set_error(ICCG_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
        }
        c->graph_iters = iters;
    }
    HIP_CHECK(hipGraphLaunch(c->graph, c->work));
    return ICCG_OK;
}

int install_factor(iccg_ctx *c) {
    // slot values and 1/L_ii from the lower-triangle factor in c->lval
    const int blocks = 1024;
    for (DevSweep *s : {&c->fwd, &c->bwd}) {
        if (c->fp32()) {
            if (!s->sval32.p) ICCG_CHECK(s->sval32.alloc(static_cast<size_t>(s->nslots)));
            hipLaunchKernelGGL(k_fill_slots<float>, dim3(blocks), dim3(256), 0, c->work,
                               s->nslots, s->ssrc.p, c->lval.p, s->sval32.p);
        } else {
            if (!s->sval64.p) ICCG_CHECK(s->sval64.alloc(static_cast<size_t>(s->nslots)));
            hipLaunchKernelGGL(k_fill_slots<double>, dim3(blocks), dim3(256), 0, c->work,
                               s->nslots, s->ssrc.p, c->lval.p, s->sval64.p);
        }
        DevWide &w = s->wide;
        if (w.nwide > 0) {
            if (c->fp32()) {
                if (!w.sval32.p) ICCG_CHECK(w.sval32.alloc(static_cast<size_t>(w.nslots)));
                hipLaunchKernelGGL(k_fill_slots<float>, dim3(blocks), dim3(256), 0, c->work,
                                   w.nslots, w.ssrc.p, c->lval.p, w.sval32.p);
            } else {
                if (!w.sval64.p) ICCG_CHECK(w.sval64.alloc(static_cast<size_t>(w.nslots)));
                hipLaunchKernelGGL(k_fill_slots<double>, dim3(blocks), dim3(256), 0, c->work,
                                   w.nslots, w.ssrc.p, c->lval.p, w.sval64.p);
            }
        }
    }
    if (c->fp32())
        hipLaunchKernelGGL(k_fill_inv<float>, dim3(blocks), dim3(256), 0, c->work, c->n,
                           c->dpos.p, c->lval.p, c->inv32.p);
    else
        hipLaunchKernelGGL(k_fill_inv<double>, dim3(blocks), dim3(256), 0, c->work, c->n,
                           c->dpos.p, c->lval.p, c->inv64.p);
    HIP_CHECK(hipGetLastError());
    c->has_factor = true;
    return ICCG_OK;
}

int upload_sweep(iccg_ctx *c, const SweepPlan &plan, DevSweep &d) {
    d.ntasks = static_cast<int>(plan.task_chunk_ptr.size()) - 1;
    d.nslots = static_cast<long long>(plan.slot_col.size());
    d.max_depth = plan.max_depth;
    d.max_width = plan.max_width;
    auto tier = [](int w) { return w <= 4 ? 4 : w <= 6 ? 6 : w <= 8 ? 8 : w <= 16 ? 16 : w <= 28 ? 28 : 32; };
    d.kmax = tier(plan.max_width);
    d.color_task_ptr = plan.color_task_ptr;
    // the register tier of each color's launch follows the widest row of
    // that color (in color-major order a row's lower entries grow with its
    // color, so early forward colors need few slots); every tier computes
    // the same terms in the same order
    const int ncol = static_cast<int>(plan.color_task_ptr.size()) - 1;
    d.color_kmax.assign(std::max(ncol, 0), 4);
    for (int col = 0; col < ncol; ++col) {
        int w = 0;
        for (int t = plan.color_task_ptr[col]; t < plan.color_task_ptr[col + 1]; ++t)
            for (int q = plan.task_chunk_ptr[t]; q < plan.task_chunk_ptr[t + 1]; ++q)
                w = std::max(w, plan.chunks[q].width());
        d.color_kmax[col] = tier(w);
    }
    ICCG_CHECK(d.tasks.upload(plan.tasks.data(), plan.tasks.size(), c->work));
    d.ndeps = static_cast<long long>(plan.deps.size());
    ICCG_CHECK(d.deps.upload(plan.deps.data(), plan.deps.size(), c->work));
    ICCG_CHECK(d.wg_task.upload(plan.wg_task.data(), plan.wg_task.size(), c->work));
    ICCG_CHECK(d.flag_loc.alloc(std::max(d.ntasks, 1)));
    ICCG_CHECK(d.flag_rem.alloc(std::max(d.ntasks, 1)));
    ICCG_CHECK(d.epoch.alloc(1));
    HIP_CHECK(hipMemsetAsync(d.flag_loc.p, 0, sizeof(int) * std::max(d.ntasks, 1), c->work));
    HIP_CHECK(hipMemsetAsync(d.flag_rem.p, 0, sizeof(int) * std::max(d.ntasks, 1), c->work));
    HIP_CHECK(hipMemsetAsync(d.epoch.p, 0, sizeof(int), c->work));
    d.remote_tasks = plan.remote_tasks;
    d.exported_rows = plan.exported_rows;
    ICCG_CHECK(d.chunks.upload(plan.chunks.data(), plan.chunks.size(), c->work));
    ICCG_CHECK(d.meta.upload(plan.meta.data(), plan.meta.size(), c->work));
    ICCG_CHECK(d.scol.upload(plan.slot_col.data(), plan.slot_col.size(), c->work));
    ICCG_CHECK(d.ssrc.upload(plan.slot_src.data(), plan.slot_src.size(), c->work));
    return ICCG_OK;
}

int upload_wide(iccg_ctx *c, const WidePlan &w, DevWide &d) {
    d.nwide = static_cast<int>(w.task.size());
    d.color_ptr = w.color_ptr;
    if (d.nwide == 0) return ICCG_OK;
    d.nslots = static_cast<long long>(w.slot_col.size());
    ICCG_CHECK(d.task.upload(w.task.data(), w.task.size(), c->work));
    ICCG_CHECK(d.piece_ptr.upload(w.piece_ptr.data(), w.piece_ptr.size(), c->work));
    ICCG_CHECK(d.pieces.upload(w.pieces.data(), w.pieces.size(), c->work));
    ICCG_CHECK(d.subs.upload(w.subs.data(), w.subs.size(), c->work));
    ICCG_CHECK(d.wmeta.upload(w.wmeta.data(), w.wmeta.size(), c->work));
    ICCG_CHECK(d.wlev.upload(w.wlev.data(), w.wlev.size(), c->work));
    ICCG_CHECK(d.scol.upload(w.slot_col.data(), w.slot_col.size(), c->work));
    ICCG_CHECK(d.ssrc.upload(w.slot_src.data(), w.slot_src.size(), c->work));
    return ICCG_OK;
}

// Host-only checks and schedule construction (no HIP call).
struct HostSetup {
    std::vector<int> dpos, tpos;
    SweepPlan fwd, bwd;
    SellMatrix sell;
    int max_block = 0;
};

int validate(int n, const int *rowptr, const int *col, const double *val, int nblocks,
             const int *block_ptr, int ncolors, const int *color_ptr, int pack_rows,
             HostSetup &hs) {
    if (n < 1 || !rowptr || !col || !val) return set_error(ICCG_EINVAL, "need n >= 1 and a CSR matrix");
    if (rowptr[0] != 0) return set_error(ICCG_EPATTERN, "rowptr[0] != 0");
    for (int i = 0; i < n; ++i)
        if (rowptr[i + 1] < rowptr[i]) return set_error(ICCG_EPATTERN, "rowptr not monotone");
    const int nnz = rowptr[n];
    std::vector<int> &dpos = hs.dpos, &tpos = hs.tpos;
    dpos.assign(n, -1);
    tpos.assign(nnz, -1);
    for (int i = 0; i < n; ++i) {
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            if (col[k] < 0 || col[k] >= n) return set_error(ICCG_EPATTERN, "column index out of range");
            if (k > rowptr[i] && col[k] <= col[k - 1])
                return set_error(ICCG_EPATTERN, "columns not strictly ascending in row " + std::to_string(i));
            if (col[k] == i) dpos[i] = k;
            if (!std::isfinite(val[k])) return set_error(ICCG_EINVAL, "non-finite matrix value");
        }
        if (dpos[i] < 0) return set_error(ICCG_EPATTERN, "diagonal missing in row " + std::to_string(i));
    }
    for (int i = 0; i < n; ++i)
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            const int j = col[k];
            const int *lo = col + rowptr[j], *hi = col + rowptr[j + 1];
            const int *f = std::lower_bound(lo, hi, i);
            if (f == hi || *f != i) return set_error(ICCG_EPATTERN, "pattern is not symmetric");
            tpos[k] = static_cast<int>(f - col);
        }
    // ordering
    if (nblocks < 1 || ncolors < 1 || !block_ptr || !color_ptr)
        return set_error(ICCG_EBADORDER, "need nblocks, ncolors >= 1 and block_ptr, color_ptr");
    if (block_ptr[0] != 0 || block_ptr[nblocks] != n) return set_error(ICCG_EBADORDER, "block_ptr must run from 0 to n");
    if (color_ptr[0] != 0 || color_ptr[ncolors] != nblocks)
        return set_error(ICCG_EBADORDER, "color_ptr must run from 0 to nblocks");
    for (int b = 0; b < nblocks; ++b) {
        if (block_ptr[b + 1] <= block_ptr[b]) return set_error(ICCG_EBADORDER, "empty or reversed block");
        hs.max_block = std::max(hs.max_block, block_ptr[b + 1] - block_ptr[b]);
    }
    for (int k = 0; k < ncolors; ++k)
        if (color_ptr[k + 1] <= color_ptr[k]) return set_error(ICCG_EBADORDER, "empty or reversed color");
    std::vector<int> blk(n), colr(nblocks);
    for (int b = 0; b < nblocks; ++b)
        for (int i = block_ptr[b]; i < block_ptr[b + 1]; ++i) blk[i] = b;
    for (int k = 0; k < ncolors; ++k)
        for (int b = color_ptr[k]; b < color_ptr[k + 1]; ++b) colr[b] = k;
    for (int i = 0; i < n; ++i)
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            const int bi = blk[i], bj = blk[col[k]];
            if (bi != bj && colr[bi] == colr[bj])
                return set_error(ICCG_EBADORDER, "blocks " + std::to_string(bi) + " and " +
                                                     std::to_string(bj) + " share an edge and a color");
        }
    ICCG_CHECK(build_sweep_plan(true, n, rowptr, col, tpos.data(), nblocks, block_ptr, ncolors,
                                color_ptr, pack_rows, hs.fwd));
    ICCG_CHECK(build_sweep_plan(false, n, rowptr, col, tpos.data(), nblocks, block_ptr, ncolors,
                                color_ptr, pack_rows, hs.bwd));
    ICCG_CHECK(build_sell(n, rowptr, col, val, block_ptr, ncolors, color_ptr, hs.sell));
    return ICCG_OK;
}

int upload_setup(iccg_ctx *c, int n, const int *rowptr, const int *col, const double *val,
                 int nblocks, int ncolors, HostSetup &hs) {
    const int nnz = rowptr[n];
    c->n = n;
    c->nnz = nnz;
    c->nnz_lower = (nnz - n) / 2;
    c->nblocks = nblocks;
    c->ncolors = ncolors;
    c->max_block = hs.max_block;
    c->h_rowptr.assign(rowptr, rowptr + n + 1);
    c->h_col.assign(col, col + nnz);
    c->h_val.assign(val, val + nnz);
    c->h_dpos = hs.dpos;

    hipStream_t s = c->work;
    ICCG_CHECK(c->rowptr.upload(rowptr, n + 1, s));
    ICCG_CHECK(c->col.upload(col, nnz, s));
    ICCG_CHECK(c->val.upload(val, nnz, s));
    ICCG_CHECK(c->dpos.upload(hs.dpos.data(), n, s));
    ICCG_CHECK(c->tpos.upload(hs.tpos.data(), nnz, s));
    if (c->opt.sweep_launch == 0 && c->opt.wide_blocks) {
        for (SweepPlan *P : {&hs.fwd, &hs.bwd}) {
            WidePlan wp;
            ICCG_CHECK(build_wide_plan(*P, n, rowptr, col, hs.tpos.data(), ncolors,
                                       64 * wide_waves(P->max_width), wp));
            ICCG_CHECK(upload_wide(c, wp, P == &hs.fwd ? c->fwd.wide : c->bwd.wide));
        }
    }
    ICCG_CHECK(upload_sweep(c, hs.fwd, c->fwd));
    ICCG_CHECK(upload_sweep(c, hs.bwd, c->bwd));
    // hybrid sweeps: the trailing colors (in forward order) holding at most
    // kFlowTailTasks tasks together, if there are at least two of them
    {
        int tail = c->ncolors, total = 0;
        while (tail > 0) {
            const int t = c->fwd.color_task_ptr[tail] - c->fwd.color_task_ptr[tail - 1];
            if (total + t > (c->opt.flow_tail > 0 ? c->opt.flow_tail : kFlowTailTasks)) break;
            total += t;
            --tail;
        }
        c->flow_tail = (c->ncolors - tail >= 2) ? tail : c->ncolors;
    }
    ICCG_CHECK(c->lval.alloc(nnz));
    if (c->fp32()) {
        ICCG_CHECK(c->inv32.alloc(n));
        ICCG_CHECK(c->y32.alloc(n));
    } else {
        ICCG_CHECK(c->inv64.alloc(n));
    }
    ICCG_CHECK(c->y64.alloc(n));
    for (DevArray<double> *v : {&c->x, &c->r, &c->z, &c->q, &c->b, &c->p})
        ICCG_CHECK(v->alloc(n));

    c->nslices = static_cast<int>(hs.sell.slice_off.size());
    {
        // padded to whole wavefronts: a wavefront loads its records at once
        const int nrec = (c->nslices + kSpmvMaxSlicesPerWave - 1) / kSpmvMaxSlicesPerWave * kSpmvMaxSlicesPerWave;
        std::vector<int4> rec(std::max(nrec, kSpmvMaxSlicesPerWave), make_int4(0, 0, 0, 0));
        for (int lg = 0; lg < c->nslices; ++lg) {
            const int sl = hs.sell.order[lg];
            rec[lg] = make_int4(sl, hs.sell.slice_off[sl], hs.sell.slice_width[sl], 0);
        }
        ICCG_CHECK(c->sell_rec.upload(rec.data(), rec.size(), s));
    }
    ICCG_CHECK(c->sell_order.upload(hs.sell.order.data(), hs.sell.order.size(), s));
    ICCG_CHECK(c->sell_col.upload(hs.sell.col.data(), hs.sell.col.size(), s));
    ICCG_CHECK(c->sell_val.upload(hs.sell.val.data(), hs.sell.val.size(), s));
    // grids are multiples of 8 so the XCD remap spreads whole ranges
    auto round8 = [](int g) { return std::max(8, (g + 7) / 8 * 8); };
    int wmax = 0;
    for (int w : hs.sell.slice_width) wmax = std::max(wmax, w);
    c->sell_wmax = wmax <= 8 ? 8 : wmax <= 16 ? 16 : 32;
    // one wavefront per spmv_slices_per_wave(wmax) slices, in launch order
    const int spw = spmv_slices_per_wave(c->sell_wmax);
    c->spmv_blocks = (c->nslices + spw - 1) / spw;
    c->vec_blocks = round8(grid_for(n, kVecThreads, kMaxVecBlocks));
    const int np = std::max({c->spmv_blocks, c->vec_blocks, c->bwd.ntasks, c->fwd.ntasks, 1});
    ICCG_CHECK(c->part.alloc(np));
    ICCG_CHECK(c->part_rr.alloc(std::max(c->fwd.ntasks, 1)));
    ICCG_CHECK(c->scal.alloc(1));
    ICCG_CHECK(c->dint.alloc(1));
    ICCG_CHECK(c->sweep_err.alloc(1));
    HIP_CHECK(hipMemsetAsync(c->sweep_err.p, 0, sizeof(int), s));
    ICCG_CHECK(c->hist.alloc(1));
    HIP_CHECK(hipStreamSynchronize(s));
    return ICCG_OK;
}

int check_ctx(iccg_ctx *c) {
    if (!c) return set_error(ICCG_EINVAL, "null context");
    return ICCG_OK;
}

int read_scalars(iccg_ctx *c) {
    HIP_CHECK(hipMemcpyAsync(c->h_scal, c->scal.p, sizeof(DevScalars), hipMemcpyDeviceToHost, c->work));
    HIP_CHECK(hipMemcpyAsync(&c->h_err, c->sweep_err.p, sizeof(int), hipMemcpyDeviceToHost, c->work));
    HIP_CHECK(hipStreamSynchronize(c->work));
    return report_sweep_err(c, c->h_err);
}

// partial sums of (a, b) into part, then the fixed-order total
int enqueue_dot(iccg_ctx *c, const double *a, const double *b, int op, double *out) {
    hipLaunchKernelGGL(k_dot, dim3(c->vec_blocks), dim3(kVecThreads), 0, c->work, c->n, a, b, c->part.p);
    HIP_CHECK(hipGetLastError());
    return launch_reduce(c, c->vec_blocks, op, out);
}

int solve_impl(iccg_ctx *c, const double *b, double *x, double tol, int maxit, int *iters,
               double *relres, double *relres_true) {
    if (!b || !x) return set_error(ICCG_EINVAL, "null b or x");
    if (!(tol >= 0.0) || maxit < 0) return set_error(ICCG_EINVAL, "need tol >= 0 and maxit >= 0");
    if (!c->has_factor) return set_error(ICCG_ESTATE, "no factor: call ic0_factor or iccg_set_factor first");
    ICCG_CHECK(flow_guard(c, 2LL * maxit + 64));
    const int n = c->n;
    hipStream_t s = c->work;
    const int hist_cap = maxit + 1;
    if (c->hist.count < static_cast<size_t>(hist_cap)) {
        ICCG_CHECK(c->hist.alloc(hist_cap));
        if (c->graph) {
            HIP_CHECK(hipGraphExecDestroy(c->graph));
            c->graph = nullptr;
        }
    }
    HIP_CHECK(hipEventRecord(c->ev_t0, s));
    HIP_CHECK(hipMemcpyAsync(c->b.p, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    HIP_CHECK(hipMemcpyAsync(c->x.p, x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(64), 0, s, c->scal.p, tol, maxit, hist_cap);
    HIP_CHECK(hipGetLastError());
    ICCG_CHECK(enqueue_dot(c, c->b.p, c->b.p, OP_BNORM, nullptr));
    // r = b - A x, stopping test on the initial residual
    ICCG_CHECK(launch_spmv(c, SP_RESID, c->x.p, c->r.p, c->b.p, nullptr));
    ICCG_CHECK(launch_reduce(c, c->spmv_blocks, OP_INIT_RR, nullptr));
    // z = M^{-1} r, rho = (r, z); p = 0 and beta = 0 make the first update p = z
    CgArgs init = no_cg();
    init.sc = c->scal.p;
    ICCG_CHECK((launch_sweep<true, SW_APPLY>(c, c->r.p, ytmp(c), init)));
    init.rdot = c->r.p;
    init.part = c->part.p;
    ICCG_CHECK((launch_sweep<false, SW_DOT_BWD>(c, ytmp(c), c->z.p, init)));
    ICCG_CHECK(launch_reduce(c, c->bwd.ntasks, OP_RHO, nullptr));
    hipLaunchKernelGGL(k_fill, dim3(c->vec_blocks), dim3(kVecThreads), 0, s, n, c->p.p, 0.0);
    HIP_CHECK(hipGetLastError());
    ICCG_CHECK(read_scalars(c));
    const int batch = std::max(1, c->opt.check_every);
    long long j = 1;
    while (c->h_scal->done == DONE_RUNNING) {
        if (c->prof) {
            // instrumented: one eager iteration at a time, events harvested
            ICCG_CHECK(enqueue_iteration(c, j));
            j += 1;
            ICCG_CHECK(read_scalars(c));
            c->prof->harvest();
        } else {
            ICCG_CHECK(run_batch(c, j, batch));
            j += batch;
            ICCG_CHECK(read_scalars(c));
        }
    }
    // the last iteration's x step, then the true residual
    hipLaunchKernelGGL(k_axpy_alpha, dim3(c->vec_blocks), dim3(kVecThreads), 0, s, n, c->x.p, c->p.p,
                       c->scal.p);
    HIP_CHECK(hipGetLastError());
    ICCG_CHECK(launch_spmv(c, SP_RESID, c->x.p, c->q.p, c->b.p, nullptr));
    ICCG_CHECK(launch_reduce(c, c->spmv_blocks, OP_TRUE, nullptr));
    HIP_CHECK(hipMemcpyAsync(x, c->x.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    HIP_CHECK(hipEventRecord(c->ev_t1, s));
    ICCG_CHECK(read_scalars(c));
    ICCG_CHECK(check_sweep_err(c));
    float ms = 0.0f;
    HIP_CHECK(hipEventElapsedTime(&ms, c->ev_t0, c->ev_t1));
    c->last_ms = ms;
    const DevScalars &h = *c->h_scal;
    c->last_iters = h.iter;
    c->last_hist = std::min(h.iter + 1, hist_cap);
    if (iters) *iters = h.iter;
    if (relres) *relres = h.relres;
    if (relres_true) *relres_true = h.relres_true;
    if (h.done == DONE_CONVERGED) return ICCG_OK;
    if (h.done == DONE_NAN) return set_error(ICCG_ENAN, "CG breakdown: (p, Ap) <= 0 or a non-finite scalar");
    return set_error(ICCG_ENOCONV, "maxit reached at relres " + std::to_string(h.relres));
}

// ---------------------------------------------------------------------------
// blocks of right-hand sides: k columns of n (column-major, ld = n), one
// independent CG per column sharing every read of the matrix and the factor
// ---------------------------------------------------------------------------
constexpr int kMaxCols = 16;

// One color of a sweep for every column: workgroups of k wavefronts.
template <typename F, bool FWD, int MODE>
int launch_sweep_cols_t(iccg_ctx *c, int k, const void *in, void *out, const CgArgs &cg, int part_ld) {
    using TIn = typename std::conditional<FWD, double, F>::type;
    using TOut = typename std::conditional<FWD, F, double>::type;
    DevSweep &d = FWD ? c->fwd : c->bwd;
    const SweepArgs<F> a = sweep_args<F>(c, d);
    const TIn *pin = static_cast<const TIn *>(in);
    TOut *pout = static_cast<TOut *>(out);
    const int ld = c->n;
    for (int step = 0; step < c->ncolors; ++step) {
        const int col = FWD ? step : c->ncolors - 1 - step;
        const int t0 = d.color_task_ptr[col], t1 = d.color_task_ptr[col + 1];
        if (t1 == t0) continue;
        const dim3 grid(t1 - t0, (k + kColWaves - 1) / kColWaves), block(64 * std::min(k, kColWaves));
#define COLS_ARGS a.tasks, a.chunks, a.meta, a.scol, a.sval, a.inv, t0, t1 - t0, pin, pout, cg, ld, part_ld, k
        switch (d.color_kmax[col]) {
            case 4: hipLaunchKernelGGL((k_sweep_cols<F, FWD, 4, MODE, TIn, TOut>), grid, block, 0, c->work, COLS_ARGS); break;
            case 6: hipLaunchKernelGGL((k_sweep_cols<F, FWD, 6, MODE, TIn, TOut>), grid, block, 0, c->work, COLS_ARGS); break;
            case 8: hipLaunchKernelGGL((k_sweep_cols<F, FWD, 8, MODE, TIn, TOut>), grid, block, 0, c->work, COLS_ARGS); break;
            case 16: hipLaunchKernelGGL((k_sweep_cols<F, FWD, 16, MODE, TIn, TOut>), grid, block, 0, c->work, COLS_ARGS); break;
            case 28: hipLaunchKernelGGL((k_sweep_cols<F, FWD, 28, MODE, TIn, TOut>), grid, block, 0, c->work, COLS_ARGS); break;
            default: hipLaunchKernelGGL((k_sweep_cols<F, FWD, 32, MODE, TIn, TOut>), grid, block, 0, c->work, COLS_ARGS); break;
        }
#undef COLS_ARGS
        HIP_CHECK(hipGetLastError());
    }
    return ICCG_OK;
}

template <bool FWD, int MODE>
int launch_sweep_cols(iccg_ctx *c, int k, const void *in, void *out, const CgArgs &cg, int part_ld) {
    return c->fp32() ? launch_sweep_cols_t<float, FWD, MODE>(c, k, in, out, cg, part_ld)
                     : launch_sweep_cols_t<double, FWD, MODE>(c, k, in, out, cg, part_ld);
}

int launch_spmv_cols(iccg_ctx *c, int k, int mode, const double *x, double *y, const double *b,
                     const DevScalars *sc, double *part, int part_ld) {
    const dim3 grid(c->spmv_blocks, (k + kColWaves - 1) / kColWaves), block(64 * std::min(k, kColWaves));
    const int ld = c->n;
#define SPMVC_ARGS c->n, c->nslices, c->sell_rec.p, c->sell_col.p, c->sell_val.p, x, y, b, part, sc, ld, part_ld, k
#define SPMVC_W(M)                                                                                    \
    switch (c->sell_wmax) {                                                                           \
        case 8: hipLaunchKernelGGL((k_spmv_cols<M, 8>), grid, block, 0, c->work, SPMVC_ARGS); break;   \
        case 16: hipLaunchKernelGGL((k_spmv_cols<M, 16>), grid, block, 0, c->work, SPMVC_ARGS); break; \
        default: hipLaunchKernelGGL((k_spmv_cols<M, 32>), grid, block, 0, c->work, SPMVC_ARGS); break; \
    }
    if (mode == SP_PLAIN) {
        SPMVC_W(SP_PLAIN)
    } else {
        SPMVC_W(SP_RESID)
    }
#undef SPMVC_W
#undef SPMVC_ARGS
    HIP_CHECK(hipGetLastError());
    return ICCG_OK;
}

int multi_part_ld(const iccg_ctx *c) { return static_cast<int>(c->part.count); }
void *mytmp(iccg_ctx *c) { return c->fp32() ? static_cast<void *>(c->my32.p) : c->my64.p; }

// Work buffers for k columns (kept for later calls with at most as many).
int ensure_multi(iccg_ctx *c, int k) {
    if (!c->h_mscal)
        HIP_CHECK(hipHostMalloc(reinterpret_cast<void **>(&c->h_mscal), sizeof(DevScalars) * kMaxCols,
                                hipHostMallocDefault));
    if (k <= c->mk) return ICCG_OK;
    const size_t nk = static_cast<size_t>(c->n) * k;
    for (DevArray<double> *v : {&c->mx, &c->mr, &c->mz, &c->mp, &c->mq, &c->mb}) ICCG_CHECK(v->alloc(nk));
    if (c->fp32()) ICCG_CHECK(c->my32.alloc(nk));
    else ICCG_CHECK(c->my64.alloc(nk));
    const size_t np = static_cast<size_t>(multi_part_ld(c));
    ICCG_CHECK(c->mpart.alloc(np * k));
    ICCG_CHECK(c->mpart_rr.alloc(np * k));
    ICCG_CHECK(c->mscal.alloc(k));
    c->mk = k;
    return ICCG_OK;
}

int launch_reduce_cols(iccg_ctx *c, int k, const double *part, int np, int op, double *out) {
    hipLaunchKernelGGL(k_reduce, dim3(k), dim3(kReduceThreads), 0, c->work, part, np, c->mscal.p, op, out,
                       c->mhist.p, multi_part_ld(c), c->mhist_cap);
    HIP_CHECK(hipGetLastError());
    return ICCG_OK;
}

// One CG iteration of every column (the single-vector iteration's kernels,
// column by column; stopped columns skip their work).
int enqueue_iteration_multi(iccg_ctx *c, int k) {
    const int pld = multi_part_ld(c);
    DevScalars *sc = c->mscal.p;
    hipLaunchKernelGGL(k_update_p_cols, dim3(c->nslices, k), dim3(64), 0, c->work, c->n, c->nslices,
                       c->sell_order.p, c->mx.p, c->mp.p, c->mz.p, sc, c->n);
    HIP_CHECK(hipGetLastError());
    ICCG_CHECK(launch_spmv_cols(c, k, SP_PLAIN, c->mp.p, c->mq.p, nullptr, sc, c->mpart.p, pld));
    ICCG_CHECK(launch_reduce_cols(c, k, c->mpart.p, c->spmv_blocks, OP_ALPHA, nullptr));
    CgArgs f = no_cg();
    f.r = c->mr.p;
    f.q = c->mq.p;
    f.part = c->mpart_rr.p;
    f.sc = sc;
    ICCG_CHECK((launch_sweep_cols<true, SW_CG_FWD>(c, k, nullptr, mytmp(c), f, pld)));
    CgArgs g = no_cg();
    g.rdot = c->mr.p;
    g.part = c->mpart.p;
    g.sc = sc;
    ICCG_CHECK((launch_sweep_cols<false, SW_DOT_BWD>(c, k, mytmp(c), c->mz.p, g, pld)));
    hipLaunchKernelGGL(k_reduce_rr_beta, dim3(k), dim3(kReduceThreads), 0, c->work, c->mpart_rr.p,
                       c->fwd.ntasks, c->mpart.p, c->bwd.ntasks, sc, c->mhist.p, pld, c->mhist_cap);
    HIP_CHECK(hipGetLastError());
    return ICCG_OK;
}

int run_batch_multi(iccg_ctx *c, int k, int iters) {
    if (!c->opt.use_graph) {
        for (int j = 0; j < iters; ++j) ICCG_CHECK(enqueue_iteration_multi(c, k));
        return ICCG_OK;
    }
    if (!c->mgraph || c->mgraph_iters != iters || c->mgraph_k != k) {
        if (c->mgraph) {
            HIP_CHECK(hipGraphExecDestroy(c->mgraph));
            c->mgraph = nullptr;
        }
        HIP_CHECK(hipStreamBeginCapture(c->work, hipStreamCaptureModeThreadLocal));
        int st = ICCG_OK;
        for (int j = 0; j < iters && st == ICCG_OK; ++j) st = enqueue_iteration_multi(c, k);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c->work, &g);
        if (st != ICCG_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return set_error(ICCG_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(&c->mgraph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            c->mgraph = nullptr;
            return set_error(ICCG_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
        }
        c->mgraph_iters = iters;
        c->mgraph_k = k;
    }
    HIP_CHECK(hipGraphLaunch(c->mgraph, c->work));
    return ICCG_OK;
}

int read_mscalars(iccg_ctx *c, int k) {
    HIP_CHECK(hipMemcpyAsync(c->h_mscal, c->mscal.p, sizeof(DevScalars) * k, hipMemcpyDeviceToHost, c->work));
    HIP_CHECK(hipStreamSynchronize(c->work));
    return ICCG_OK;
}

int solve_multi_impl(iccg_ctx *c, int k, const double *B, double *X, double tol, int maxit, int *iters,
                     double *relres, double *relres_true) {
    if (k < 1 || k > kMaxCols) return set_error(ICCG_EINVAL, "need 1 <= k <= 16 right-hand sides");
    if (!B || !X) return set_error(ICCG_EINVAL, "null B or X");
    if (!(tol >= 0.0) || maxit < 0) return set_error(ICCG_EINVAL, "need tol >= 0 and maxit >= 0");
    if (!c->has_factor) return set_error(ICCG_ESTATE, "no factor: call ic0_factor or iccg_set_factor first");
    ICCG_CHECK(ensure_multi(c, k));
    const int hist_cap = maxit + 1;
    if (c->mhist.count < static_cast<size_t>(hist_cap) * k || c->mhist_cap != hist_cap) {
        if (c->mhist.count < static_cast<size_t>(hist_cap) * k)
            ICCG_CHECK(c->mhist.alloc(static_cast<size_t>(hist_cap) * k));
        c->mhist_cap = hist_cap;
        if (c->mgraph) {
            HIP_CHECK(hipGraphExecDestroy(c->mgraph));
            c->mgraph = nullptr;
        }
    }
    const int n = c->n;
    const size_t nk = static_cast<size_t>(n) * k;
    const int pld = multi_part_ld(c);
    hipStream_t s = c->work;
    HIP_CHECK(hipEventRecord(c->ev_t0, s));
    HIP_CHECK(hipMemcpyAsync(c->mb.p, B, sizeof(double) * nk, hipMemcpyDeviceToDevice, s));
    HIP_CHECK(hipMemcpyAsync(c->mx.p, X, sizeof(double) * nk, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_init_scalars, dim3(k), dim3(64), 0, s, c->mscal.p, tol, maxit, hist_cap);
    hipLaunchKernelGGL(k_dot_cols, dim3(c->vec_blocks, k), dim3(kVecThreads), 0, s, n, c->mb.p, c->mb.p,
                       c->mpart.p, n, pld);
    HIP_CHECK(hipGetLastError());
    ICCG_CHECK(launch_reduce_cols(c, k, c->mpart.p, c->vec_blocks, OP_BNORM, nullptr));
    // r = b - A x, stopping test on the initial residual
    ICCG_CHECK(launch_spmv_cols(c, k, SP_RESID, c->mx.p, c->mr.p, c->mb.p, nullptr, c->mpart.p, pld));
    ICCG_CHECK(launch_reduce_cols(c, k, c->mpart.p, c->spmv_blocks, OP_INIT_RR, nullptr));
    // z = M^{-1} r, rho = (r, z); p = 0 and beta = 0 make the first update p = z
    CgArgs init = no_cg();
    init.sc = c->mscal.p;
    ICCG_CHECK((launch_sweep_cols<true, SW_APPLY>(c, k, c->mr.p, mytmp(c), init, pld)));
    init.rdot = c->mr.p;
    init.part = c->mpart.p;
    ICCG_CHECK((launch_sweep_cols<false, SW_DOT_BWD>(c, k, mytmp(c), c->mz.p, init, pld)));
    ICCG_CHECK(launch_reduce_cols(c, k, c->mpart.p, c->bwd.ntasks, OP_RHO, nullptr));
    hipLaunchKernelGGL(k_fill, dim3(c->vec_blocks), dim3(kVecThreads), 0, s, static_cast<int>(nk), c->mp.p, 0.0);
    HIP_CHECK(hipGetLastError());
    ICCG_CHECK(read_mscalars(c, k));
    auto running = [&]() {
        for (int j = 0; j < k; ++j)
            if (c->h_mscal[j].done == DONE_RUNNING) return true;
        return false;
    };
    const int batch = std::max(1, c->opt.check_every);
    while (running()) {
        ICCG_CHECK(run_batch_multi(c, k, batch));
        ICCG_CHECK(read_mscalars(c, k));
    }
    hipLaunchKernelGGL(k_axpy_alpha_cols, dim3(c->vec_blocks, k), dim3(kVecThreads), 0, s, n, c->mx.p, c->mp.p,
                       c->mscal.p, n);
    HIP_CHECK(hipGetLastError());
    ICCG_CHECK(launch_spmv_cols(c, k, SP_RESID, c->mx.p, c->mq.p, c->mb.p, nullptr, c->mpart.p, pld));
    ICCG_CHECK(launch_reduce_cols(c, k, c->mpart.p, c->spmv_blocks, OP_TRUE, nullptr));
    HIP_CHECK(hipMemcpyAsync(X, c->mx.p, sizeof(double) * nk, hipMemcpyDeviceToDevice, s));
    HIP_CHECK(hipEventRecord(c->ev_t1, s));
    ICCG_CHECK(read_mscalars(c, k));
    float ms = 0.0f;
    HIP_CHECK(hipEventElapsedTime(&ms, c->ev_t0, c->ev_t1));
    c->last_ms = ms;
    int status = ICCG_OK;
    for (int j = 0; j < k; ++j) {
        const DevScalars &h = c->h_mscal[j];
        if (iters) iters[j] = h.iter;
        if (relres) relres[j] = h.relres;
        if (relres_true) relres_true[j] = h.relres_true;
        if (h.done == DONE_NAN) status = ICCG_ENAN;
        else if (h.done != DONE_CONVERGED && status == ICCG_OK) status = ICCG_ENOCONV;
    }
    if (status == ICCG_ENAN) return set_error(ICCG_ENAN, "CG breakdown in a column: (p, Ap) <= 0 or a non-finite scalar");
    if (status == ICCG_ENOCONV) return set_error(ICCG_ENOCONV, "maxit reached in a column");
    return ICCG_OK;
}

template <typename F>
int entry(iccg_ctx *c, F &&body) {
    try {
        ICCG_CHECK(check_ctx(c));
        ICCG_CHECK(c->enter());
        const int st = body();
        const int st2 = c->leave();
        return st != ICCG_OK ? st : st2;
    } catch (const std::bad_alloc &) {
        return set_error(ICCG_ENOMEM, "host allocation failed");
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void iccg_default_options(iccg_options *opt) {
    if (!opt) return;
    opt->precision = ICCG_FP64;
    opt->stream = nullptr;
    opt->check_every = 32;
    opt->pack_rows = 64;
    opt->use_graph = 1;
    opt->sweep_launch = 0;
    opt->sweep_grid = 0;
    opt->flow_tail = 0;
    opt->wide_blocks = 1;
    opt->host_factor = 0;
    opt->fuse_turn = 1;
}

const char *iccg_strerror(int st) {
    switch (st) {
        case ICCG_OK: return "ok";
        case ICCG_EINVAL: return "invalid argument";
        case ICCG_EPATTERN: return "bad sparsity pattern";
        case ICCG_EBADORDER: return "bad block/color ordering";
        case ICCG_EBREAKDOWN: return "IC(0) breakdown";
        case ICCG_ENOCONV: return "not converged";
        case ICCG_ENAN: return "CG breakdown or non-finite value";
        case ICCG_EHIP: return "HIP runtime error";
        case ICCG_ENOMEM: return "out of memory";
        case ICCG_ESTATE: return "call out of order";
        default: return "unknown status";
    }
}

const char *iccg_last_error(void) { return g_last_error.c_str(); }

int iccg_setup(iccg_ctx **out, int n, const int *rowptr, const int *col, const double *val,
               int nblocks, const int *block_ptr, int ncolors, const int *color_ptr,
               const iccg_options *opt) {
    if (!out) return set_error(ICCG_EINVAL, "null out");
    *out = nullptr;
    try {
        std::unique_ptr<iccg_ctx> c(new iccg_ctx());
        iccg_default_options(&c->opt);
        if (opt) c->opt = *opt;
        if (c->opt.precision != ICCG_FP64 && c->opt.precision != ICCG_FP32)
            return set_error(ICCG_EINVAL, "precision must be ICCG_FP64 or ICCG_FP32");
        if (c->opt.check_every < 1) c->opt.check_every = 1;
        if (c->opt.pack_rows < 1 || c->opt.pack_rows > kChunkRows) c->opt.pack_rows = kChunkRows;
        if (c->opt.sweep_launch < 0 || c->opt.sweep_launch > 2)
            return set_error(ICCG_EINVAL, "sweep_launch must be 0, 1 or 2");
        if (c->opt.sweep_grid < 0) return set_error(ICCG_EINVAL, "sweep_grid must be >= 0");
        if (c->opt.flow_tail < 0) return set_error(ICCG_EINVAL, "flow_tail must be >= 0");
        // the single-launch sweep addresses vectors and flags through 32-bit
        // buffer ranges
        if (c->opt.sweep_launch != 0 && n >= (1 << 27))
            return set_error(ICCG_EINVAL, "the single-launch sweep needs n < 2^27");
        HostSetup hs;
        ICCG_CHECK(validate(n, rowptr, col, val, nblocks, block_ptr, ncolors, color_ptr,
                            c->opt.pack_rows, hs));
        ICCG_CHECK(iccg_block_stats(nblocks, block_ptr, ncolors, color_ptr, c->stats6));
        c->user = static_cast<hipStream_t>(c->opt.stream);
        HIP_CHECK(hipStreamCreateWithFlags(&c->work, hipStreamNonBlocking));
        int dev = 0;
        HIP_CHECK(hipGetDevice(&dev));
        c->device = dev;
        ICCG_CHECK(resolve_scratch(dev));
        HIP_CHECK(hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, dev));
        HIP_CHECK(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
        HIP_CHECK(hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
        HIP_CHECK(hipEventCreate(&c->ev_t0));
        HIP_CHECK(hipEventCreate(&c->ev_t1));
        HIP_CHECK(hipHostMalloc(reinterpret_cast<void **>(&c->h_scal), sizeof(DevScalars), hipHostMallocDefault));
        ICCG_CHECK(c->enter());
        ICCG_CHECK(upload_setup(c.get(), n, rowptr, col, val, nblocks, ncolors, hs));
        ICCG_CHECK(c->leave());
        *out = c.release();
        return ICCG_OK;
    } catch (const std::bad_alloc &) {
        return set_error(ICCG_ENOMEM, "host allocation failed in iccg_setup");
    }
}

void iccg_destroy(iccg_ctx *c) {
    if (!c) return;
    if (c->work) (void)hipStreamSynchronize(c->work);
    delete c;
}

int ic0_factor(iccg_ctx *c, int *breakdown_row) {
    return entry(c, [&]() -> int {
        if (breakdown_row) *breakdown_row = -1;
        int row = -1;
        std::vector<double> lv;
        if (c->opt.host_factor) {
            row = ic0_host(c->n, c->h_rowptr.data(), c->h_col.data(), c->h_val.data(), c->h_dpos.data(), lv);
            if (row < 0)
                HIP_CHECK(hipMemcpyAsync(c->lval.p, lv.data(), sizeof(double) * lv.size(), hipMemcpyHostToDevice,
                                         c->work));
        } else {
            // the forward sweep's schedule, color by color
            hipLaunchKernelGGL(k_fill, dim3(grid_for(c->nnz, kVecThreads, kMaxVecBlocks)), dim3(kVecThreads), 0,
                               c->work, c->nnz, c->lval.p, 0.0);
            hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, c->work, c->dint.p, INT_MAX);
            const DevSweep &d = c->fwd;
            for (int col = 0; col < c->ncolors; ++col) {
                const int t0 = d.color_task_ptr[col], t1 = d.color_task_ptr[col + 1];
                if (t1 == t0) continue;
                hipLaunchKernelGGL(k_ic0, dim3(t1 - t0), dim3(64), 0, c->work, d.tasks.p, d.chunks.p, d.meta.p,
                                   t0, t1 - t0, c->rowptr.p, c->col.p, c->val.p, c->dpos.p, c->lval.p, c->dint.p);
            }
            HIP_CHECK(hipGetLastError());
            int bad = INT_MAX;
            HIP_CHECK(hipMemcpyAsync(&bad, c->dint.p, sizeof(int), hipMemcpyDeviceToHost, c->work));
            HIP_CHECK(hipStreamSynchronize(c->work));
            row = bad == INT_MAX ? -1 : bad;
        }
        if (row >= 0) {
            c->has_factor = false;
            if (breakdown_row) *breakdown_row = row;
            return set_error(ICCG_EBREAKDOWN, "IC(0) pivot not positive at row " + std::to_string(row));
        }
        if (!c->lval0.p) ICCG_CHECK(c->lval0.alloc(c->nnz));
        HIP_CHECK(hipMemcpyAsync(c->lval0.p, c->lval.p, sizeof(double) * c->nnz, hipMemcpyDeviceToDevice, c->work));
        c->has_ic0 = true;
        ICCG_CHECK(install_factor(c));
        HIP_CHECK(hipStreamSynchronize(c->work));   // lv is released on return
        return ICCG_OK;
    });
}

int iccg_set_factor(iccg_ctx *c, const double *lvals_dev, int *bad_row) {
    return entry(c, [&]() -> int {
        if (bad_row) *bad_row = -1;
        if (!lvals_dev) return set_error(ICCG_EINVAL, "null factor");
        if (!c->lstage.p) ICCG_CHECK(c->lstage.alloc(c->nnz));
        hipLaunchKernelGGL(k_take_lower, dim3(grid_for(c->n, 256, 4096)), dim3(256), 0, c->work, c->n,
                           c->rowptr.p, c->col.p, lvals_dev, c->lstage.p);
        hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, c->work, c->dint.p, INT_MAX);
        hipLaunchKernelGGL(k_check_factor, dim3(grid_for(c->n, 256, 4096)), dim3(256), 0, c->work,
                           c->n, c->rowptr.p, c->col.p, c->dpos.p, c->lstage.p, c->dint.p);
        HIP_CHECK(hipGetLastError());
        int bad = INT_MAX;
        HIP_CHECK(hipMemcpyAsync(&bad, c->dint.p, sizeof(int), hipMemcpyDeviceToHost, c->work));
        HIP_CHECK(hipStreamSynchronize(c->work));
        if (bad != INT_MAX) {
            if (bad_row) *bad_row = bad;
            return set_error(ICCG_EBREAKDOWN, "factor rejected at row " + std::to_string(bad));
        }
        HIP_CHECK(hipMemcpyAsync(c->lval.p, c->lstage.p, sizeof(double) * c->nnz, hipMemcpyDeviceToDevice, c->work));
        return install_factor(c);
    });
}

int iccg_restore_ic0(iccg_ctx *c) {
    return entry(c, [&]() -> int {
        if (!c->has_ic0) return set_error(ICCG_ESTATE, "no IC(0) factor: call ic0_factor first");
        HIP_CHECK(hipMemcpyAsync(c->lval.p, c->lval0.p, sizeof(double) * c->nnz, hipMemcpyDeviceToDevice, c->work));
        return install_factor(c);
    });
}

int iccg_get_factor(iccg_ctx *c, double *lvals) {
    return entry(c, [&]() -> int {
        if (!lvals) return set_error(ICCG_EINVAL, "null output");
        if (!c->has_factor) return set_error(ICCG_ESTATE, "no factor");
        HIP_CHECK(hipMemcpyAsync(lvals, c->lval.p, sizeof(double) * c->nnz, hipMemcpyDeviceToHost, c->work));
        HIP_CHECK(hipStreamSynchronize(c->work));
        return ICCG_OK;
    });
}

int ic_apply(iccg_ctx *c, const double *r, double *z) {
    return entry(c, [&]() -> int {
        if (!r || !z) return set_error(ICCG_EINVAL, "null vector");
        if (r == z) return set_error(ICCG_EINVAL, "r and z must not alias");
        if (!c->has_factor) return set_error(ICCG_ESTATE, "no factor");
        ICCG_CHECK(flow_guard(c, 2));
        ICCG_CHECK((launch_sweep<true, SW_APPLY>(c, r, ytmp(c), no_cg())));
        ICCG_CHECK((launch_sweep<false, SW_APPLY>(c, ytmp(c), z, no_cg())));
        return check_sweep_err(c);
    });
}

int ic_forward(iccg_ctx *c, const double *r, double *y) {
    return entry(c, [&]() -> int {
        if (!r || !y) return set_error(ICCG_EINVAL, "null vector");
        if (!c->has_factor) return set_error(ICCG_ESTATE, "no factor");
        ICCG_CHECK(flow_guard(c, 1));
        if (c->fp32()) {
            ICCG_CHECK((launch_sweep<true, SW_APPLY>(c, r, c->y32.p, no_cg())));
            hipLaunchKernelGGL((k_convert<double, float>), dim3(c->vec_blocks), dim3(kVecThreads), 0,
                               c->work, c->n, y, c->y32.p);
            HIP_CHECK(hipGetLastError());
            return check_sweep_err(c);
        }
        if (r == y) return set_error(ICCG_EINVAL, "r and y must not alias");
        ICCG_CHECK((launch_sweep<true, SW_APPLY>(c, r, y, no_cg())));
        return check_sweep_err(c);
    });
}

int ic_backward(iccg_ctx *c, const double *y, double *z) {
    return entry(c, [&]() -> int {
        if (!y || !z) return set_error(ICCG_EINVAL, "null vector");
        if (y == z) return set_error(ICCG_EINVAL, "y and z must not alias");
        if (!c->has_factor) return set_error(ICCG_ESTATE, "no factor");
        ICCG_CHECK(flow_guard(c, 1));
        // on its own, the backward sweep's dataflow part gets its epoch here
        if (c->opt.sweep_launch == 2)
            hipLaunchKernelGGL(k_bump_epoch, dim3(1), dim3(64), 0, c->work, c->bwd.epoch.p, nullptr);
        if (c->fp32()) {
            hipLaunchKernelGGL((k_convert<float, double>), dim3(c->vec_blocks), dim3(kVecThreads), 0,
                               c->work, c->n, c->y32.p, y);
            HIP_CHECK(hipGetLastError());
            ICCG_CHECK((launch_sweep<false, SW_APPLY>(c, c->y32.p, z, no_cg())));
            return check_sweep_err(c);
        }
        ICCG_CHECK((launch_sweep<false, SW_APPLY>(c, y, z, no_cg())));
        return check_sweep_err(c);
    });
}

int iccg_spmv(iccg_ctx *c, const double *p, double *q, double *pq_host) {
    return entry(c, [&]() -> int {
        if (!p || !q || p == q) return set_error(ICCG_EINVAL, "need distinct p and q");
        ICCG_CHECK(launch_spmv(c, SP_PLAIN, p, q, nullptr, nullptr));
        if (pq_host) {
            ICCG_CHECK(launch_reduce(c, c->spmv_blocks, OP_STORE, c->b.p));
            HIP_CHECK(hipMemcpyAsync(pq_host, c->b.p, sizeof(double), hipMemcpyDeviceToHost, c->work));
            HIP_CHECK(hipStreamSynchronize(c->work));
        }
        return ICCG_OK;
    });
}

int iccg_spmv_dot_noalloc(iccg_ctx *c, const double *p, double *q, double *pq_dev) {
    return entry(c, [&]() -> int {
        if (!p || !q || !pq_dev || p == q) return set_error(ICCG_EINVAL, "need distinct p, q and a device pq");
        if (c->n > kNoAllocMaxRows || c->spmv_blocks > kNoAllocParts)
            return set_error(ICCG_EINVAL, "iccg_spmv_dot_noalloc: n = " + std::to_string(c->n) +
                                              " exceeds the static scratch (at most 2^24 rows)");
        double *part = scratch_for(c->device);
        if (!part) return set_error(ICCG_ESTATE, "static scratch not resolved for this device");
        ICCG_CHECK(launch_spmv(c, SP_PLAIN, p, q, nullptr, nullptr, part));
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kReduceThreads), 0, c->work, part, c->spmv_blocks,
                           c->scal.p, OP_STORE, pq_dev, c->hist.p, 0, 0);
        HIP_CHECK(hipGetLastError());
        return ICCG_OK;
    });
}

int iccg_dot(iccg_ctx *c, const double *a, const double *b, double *out_host) {
    return entry(c, [&]() -> int {
        if (!a || !b || !out_host) return set_error(ICCG_EINVAL, "null argument");
        ICCG_CHECK(enqueue_dot(c, a, b, OP_STORE, c->q.p));
        HIP_CHECK(hipMemcpyAsync(out_host, c->q.p, sizeof(double), hipMemcpyDeviceToHost, c->work));
        HIP_CHECK(hipStreamSynchronize(c->work));
        return ICCG_OK;
    });
}

int iccg_mpnn_smooth_probes(iccg_ctx *c, const double *z, int nprobes, double *out) {
    return entry(c, [&]() -> int {
        if (!z || !out || nprobes < 1) return set_error(ICCG_EINVAL, "need z, out and nprobes >= 1");
        if (!c->has_factor) return set_error(ICCG_ESTATE, "no factor");
        ICCG_CHECK(flow_guard(c, 2LL * nprobes));
        const int n = c->n;
        const dim3 grid(c->vec_blocks), block(kVecThreads);
        for (int i = 0; i < nprobes; ++i) {
            const double *zi = z + static_cast<size_t>(i) * n;
            double *oi = out + static_cast<size_t>(i) * n;
            hipLaunchKernelGGL(k_scale_sqrt_diag, grid, block, 0, c->work, n, c->dpos.p, c->val.p, zi, c->r.p);
            HIP_CHECK(hipGetLastError());
            ICCG_CHECK((launch_sweep<true, SW_APPLY>(c, c->r.p, ytmp(c), no_cg())));
            ICCG_CHECK((launch_sweep<false, SW_APPLY>(c, ytmp(c), c->z.p, no_cg())));
            hipLaunchKernelGGL(k_scale_sqrt_diag, grid, block, 0, c->work, n, c->dpos.p, c->val.p, c->z.p, oi);
            HIP_CHECK(hipGetLastError());
            ICCG_CHECK(enqueue_dot(c, oi, oi, OP_STORE, c->q.p));
            hipLaunchKernelGGL(k_rescale_to_norm, grid, block, 0, c->work, n, oi, c->q.p,
                               std::sqrt(static_cast<double>(n)));
            HIP_CHECK(hipGetLastError());
        }
        return check_sweep_err(c);
    });
}

int iccg_solve(iccg_ctx *c, const double *b, double *x, double tol, int maxit, int *iters,
               double *relres, double *relres_true) {
    return entry(c, [&]() -> int { return solve_impl(c, b, x, tol, maxit, iters, relres, relres_true); });
}

int iccg_solve_multi(iccg_ctx *c, int k, const double *B, double *X, double tol, int maxit, int *iters,
                     double *relres, double *relres_true) {
    return entry(c, [&]() -> int {
        return solve_multi_impl(c, k, B, X, tol, maxit, iters, relres, relres_true);
    });
}

int ic_apply_multi(iccg_ctx *c, int k, const double *R, double *Z) {
    return entry(c, [&]() -> int {
        if (k < 1 || k > kMaxCols) return set_error(ICCG_EINVAL, "need 1 <= k <= 16 columns");
        if (!R || !Z) return set_error(ICCG_EINVAL, "null block vector");
        if (R == Z) return set_error(ICCG_EINVAL, "R and Z must not alias");
        if (!c->has_factor) return set_error(ICCG_ESTATE, "no factor");
        ICCG_CHECK(ensure_multi(c, k));
        ICCG_CHECK((launch_sweep_cols<true, SW_APPLY>(c, k, R, mytmp(c), no_cg(), multi_part_ld(c))));
        ICCG_CHECK((launch_sweep_cols<false, SW_APPLY>(c, k, mytmp(c), Z, no_cg(), multi_part_ld(c))));
        return ICCG_OK;
    });
}

int iccg_spmv_multi(iccg_ctx *c, int k, const double *P, double *Q) {
    return entry(c, [&]() -> int {
        if (k < 1 || k > kMaxCols) return set_error(ICCG_EINVAL, "need 1 <= k <= 16 columns");
        if (!P || !Q || P == Q) return set_error(ICCG_EINVAL, "need distinct P and Q");
        ICCG_CHECK(ensure_multi(c, k));
        return launch_spmv_cols(c, k, SP_PLAIN, P, Q, nullptr, nullptr, c->mpart.p, multi_part_ld(c));
    });
}

int iccg_profile_solve(iccg_ctx *c, const double *b, double *x, double tol, int maxit,
                       double *out) {
    if (!out) return set_error(ICCG_EINVAL, "null output");
    Profiler prof;
    int iters = 0;
    double rr = 0.0, rt = 0.0;
    int st = entry(c, [&]() -> int {
        c->prof = &prof;
        const int r = solve_impl(c, b, x, tol, maxit, &iters, &rr, &rt);
        c->prof = nullptr;
        (void)hipStreamSynchronize(c->work);
        prof.harvest();
        return r;
    });
    if (c) c->prof = nullptr;
    out[0] = c ? c->last_ms : 0.0;
    out[1] = prof.ms[PK_SPMV];
    out[2] = prof.ms[PK_FWD];
    out[3] = prof.ms[PK_BWD];
    out[4] = out[0] - out[1] - out[2] - out[3];
    out[5] = static_cast<double>(prof.launches[PK_FWD]);
    out[6] = static_cast<double>(prof.launches[PK_BWD]);
    out[7] = static_cast<double>(prof.launches[PK_SPMV]);
    out[8] = iters;
    out[9] = rt;
    return st;
}

int iccg_residual_history(iccg_ctx *c, double *hist, int cap) {
    if (!c || !hist || cap < 0) return set_error(ICCG_EINVAL, "bad argument");
    const int k = std::min(cap, c->last_hist);
    if (k <= 0) return 0;
    hipError_t e = hipMemcpy(hist, c->hist.p, sizeof(double) * k, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return set_error(ICCG_EHIP, hipGetErrorString(e));
    return k;
}

int iccg_schedule_stats(int n, const int *rowptr, const int *col, const double *val, int nblocks,
                        const int *block_ptr, int ncolors, const int *color_ptr, int pack_rows,
                        long long *out) {
    if (!out) return set_error(ICCG_EINVAL, "null output");
    try {
        if (pack_rows < 1 || pack_rows > kChunkRows) pack_rows = kChunkRows;
        HostSetup hs;
        ICCG_CHECK(validate(n, rowptr, col, val, nblocks, block_ptr, ncolors, color_ptr, pack_rows, hs));
        int k = 0;
        for (const SweepPlan *P : {&hs.fwd, &hs.bwd}) {
            ICCG_CHECK(check_sweep_plan(*P, n, rowptr, col, ncolors, block_ptr, color_ptr));
            out[k++] = static_cast<long long>(P->task_chunk_ptr.size()) - 1;
            out[k++] = static_cast<long long>(P->chunks.size());
            out[k++] = static_cast<long long>(P->slot_col.size());
            out[k++] = P->max_depth;
            out[k++] = P->max_width;
            out[k++] = static_cast<long long>(P->deps.size());
            out[k++] = P->remote_tasks;
            out[k++] = P->exported_rows;
            out[k++] = std::count_if(P->chunks.begin(), P->chunks.end(),
                                     [](const Chunk &ch) { return !ch.jagged(); });
        }
        return ICCG_OK;
    } catch (const std::bad_alloc &) {
        return set_error(ICCG_ENOMEM, "host allocation failed");
    }
}

int iccg_get_info(iccg_ctx *c, iccg_info *info) {
    if (!c || !info) return set_error(ICCG_EINVAL, "bad argument");
    std::memset(info, 0, sizeof(*info));
    info->n = c->n;
    info->nnz = c->nnz;
    info->nnz_lower = c->nnz_lower;
    info->nblocks = c->nblocks;
    info->ncolors = c->ncolors;
    info->ntasks_fwd = c->fwd.ntasks;
    info->nchunks_fwd = static_cast<int>(c->fwd.chunks.count);
    info->max_block = c->max_block;
    info->max_depth = std::max(c->fwd.max_depth, c->bwd.max_depth);
    info->precision = c->opt.precision;
    info->has_factor = c->has_factor ? 1 : 0;
    // compulsory bytes: values + int32 columns of the strict triangle, 1/L_ii,
    // the input vector, the output vector and the CSR row pointer
    const double v = c->fp32() ? 4.0 : 8.0;
    info->sweep_bytes = (v + 4.0) * c->nnz_lower + (2.0 * v + 8.0 + 4.0) * c->n + 4.0;
    info->spmv_bytes = 12.0 * c->nnz + 20.0 * c->n + 4.0;
    info->last_solve_ms = c->last_ms;
    info->last_iters = c->last_iters;
    info->sweep_resident = c->last_resident;
    info->remote_tasks = c->fwd.remote_tasks;
    info->exported_rows = c->fwd.exported_rows;
    info->gini = c->stats6[2];
    info->bmax_over_avg = c->stats6[4];
    info->cmax_over_avg = c->stats6[5];
    return ICCG_OK;
}

}  // extern "C"
