// MI355X (gfx950) device path of block-multicolored ICCG and the C ABI in
// include/iccg.h.
//
// Per CG iteration (Section 5, IC(0)-preconditioned CG):
//   q = A'p with (p, q)                       k_spmv
//   alpha = (r, z)/(p, q)                     k_reduce
//   x += alpha p, r -= alpha q, ||r||^2       k_update_xr, k_reduce (stopping test)
//   y = L^{-1} r   (Algorithm 1)              k_sweep<forward>, one launch per color
//   z = L^{-T} y, (r, z) per task             k_sweep<backward>, one launch per color
//   beta, rho                                 k_reduce
//   p = z + beta p                            k_update_p
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

#include "iccg_internal.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

namespace iccg {

thread_local std::string g_last_error;

int set_error(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

}  // namespace iccg

using namespace iccg;

#define HIP_CHECK(expr)                                                                    \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return set_error(e_ == hipErrorOutOfMemory ? ICCG_ENOMEM : ICCG_EHIP,          \
                             std::string(#expr) + ": " + hipGetErrorString(e_));           \
    } while (0)

#define ICCG_CHECK(expr)             \
    do {                             \
        int st_ = (expr);            \
        if (st_ != ICCG_OK) return st_; \
    } while (0)

// ---------------------------------------------------------------------------
// device scalars of one CG solve
// ---------------------------------------------------------------------------
enum : int { DONE_RUNNING = 0, DONE_CONVERGED = 1, DONE_NAN = 2, DONE_MAXIT = 3 };

struct DevScalars {
    double rho;       // (r, z)
    double alpha, beta;
    double bnorm;     // ||b||
    double relres;    // ||r||/||b|| after the last update
    double relres_true;
    double tol;
    int iter;         // completed iterations
    int done;
    int maxit;
    int hist_cap;
};

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
constexpr int kMaxVecBlocks = 2048;

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
    // fixed butterfly over the 64 lanes of a wavefront
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic sum over a workgroup of kVecThreads threads; result valid in
// thread 0.
__device__ inline double block_sum(double v) {
    __shared__ double red[kVecThreads / 64];
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < kVecThreads / 64; ++k) s += red[k];
    return s;
}

__global__ __launch_bounds__(kVecThreads) void k_reduce(const double *__restrict__ part, int np,
                                                        DevScalars *sc, int op,
                                                        double *__restrict__ out,
                                                        double *__restrict__ hist) {
    if (op != OP_STORE && op != OP_TRUE && op != OP_BNORM && sc->done != DONE_RUNNING) return;
    double v = 0.0;
    for (int k = threadIdx.x; k < np; k += kVecThreads) v += part[k];
    v = block_sum(v);
    if (threadIdx.x != 0) return;
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

__global__ void k_init_scalars(DevScalars *sc, double tol, int maxit, int hist_cap) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
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
// SpMV, CSR with G lanes per row (G = 4..64, chosen from the mean row length)
// MODE 0: y = A x, partial (x, y).   MODE 1: y = b - A x, partial (y, y).
// ---------------------------------------------------------------------------
template <int G, int MODE>
__global__ __launch_bounds__(kVecThreads) void k_spmv(int n, const int *__restrict__ rowptr,
                                                      const int *__restrict__ col,
                                                      const double *__restrict__ val,
                                                      const double *__restrict__ x,
                                                      double *__restrict__ y,
                                                      const double *__restrict__ b,
                                                      double *__restrict__ part,
                                                      const DevScalars *sc) {
    if (sc && sc->done != DONE_RUNNING) return;
    constexpr int RPW = kVecThreads / G;  // rows per workgroup pass
    const int lane = threadIdx.x % G;
    const int grp = threadIdx.x / G;
    double acc = 0.0;
    for (int row0 = blockIdx.x * RPW; row0 < n; row0 += gridDim.x * RPW) {
        const int row = row0 + grp;
        double s = 0.0;
        if (row < n) {
            const int a = rowptr[row], e = rowptr[row + 1];
            for (int k = a + lane; k < e; k += G) s += val[k] * x[col[k]];
        }
        for (int off = G / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, G);
        if (lane == 0 && row < n) {
            if (MODE == 0) {
                y[row] = s;
                acc += x[row] * s;
            } else {
                const double rv = b[row] - s;
                y[row] = rv;
                acc += rv * rv;
            }
        }
    }
    const double t = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// ---------------------------------------------------------------------------
// BLAS-1 pieces of the CG step
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kVecThreads) void k_dot(int n, const double *__restrict__ a,
                                                     const double *__restrict__ b,
                                                     double *__restrict__ part) {
    double acc = 0.0;
    for (int i = blockIdx.x * kVecThreads + threadIdx.x; i < n; i += gridDim.x * kVecThreads)
        acc += a[i] * b[i];
    const double t = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(kVecThreads) void k_update_xr(int n, double *__restrict__ x,
                                                           double *__restrict__ r,
                                                           const double *__restrict__ p,
                                                           const double *__restrict__ q,
                                                           const DevScalars *sc,
                                                           double *__restrict__ part) {
    if (sc->done != DONE_RUNNING) return;
    const double alpha = sc->alpha;
    double acc = 0.0;
    for (int i = blockIdx.x * kVecThreads + threadIdx.x; i < n; i += gridDim.x * kVecThreads) {
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        acc += ri * ri;
    }
    const double t = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(kVecThreads) void k_update_p(int n, double *__restrict__ p,
                                                          const double *__restrict__ z,
                                                          const DevScalars *sc) {
    if (sc->done != DONE_RUNNING) return;
    const double beta = sc->beta;
    for (int i = blockIdx.x * kVecThreads + threadIdx.x; i < n; i += gridDim.x * kVecThreads)
        p[i] = z[i] + beta * p[i];
}

__global__ __launch_bounds__(kVecThreads) void k_copy(int n, double *__restrict__ dst,
                                                      const double *__restrict__ src,
                                                      const DevScalars *sc) {
    if (sc && sc->done != DONE_RUNNING) return;
    for (int i = blockIdx.x * kVecThreads + threadIdx.x; i < n; i += gridDim.x * kVecThreads)
        dst[i] = src[i];
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

// ---------------------------------------------------------------------------
// substitution sweep over the tasks of one color
// ---------------------------------------------------------------------------
struct SweepArgs {
    const int *task_chunk_ptr;
    const Chunk *chunks;
    const uint32_t *meta;
    const int *scol;
    const void *sval;   // F[nslots]
    const void *inv;    // F[n], 1 / L_ii
};

// FWD: y_i = (r_i - sum_{j<i} L_ij y_j) / L_ii over the rows of the color.
// !FWD: z_i = (y_i - sum_{j>i} L_ji z_j) / L_ii; with rdot != null each task
// also writes sum over its rows of rdot_i * z_i to part[task].
// TIn is the right-hand side type, TOut the solution type (read back for
// dependencies); the arithmetic is in F.
template <typename F, bool FWD, typename TIn, typename TOut>
__global__ __launch_bounds__(64) void k_sweep(SweepArgs a, int task_base,
                                              const TIn *__restrict__ in, TOut *__restrict__ out,
                                              const double *__restrict__ rdot,
                                              double *__restrict__ part, const DevScalars *sc) {
    if (sc && sc->done != DONE_RUNNING) return;
    __shared__ F ys[kChunkRows];
    const F *__restrict__ sval = static_cast<const F *>(a.sval);
    const F *__restrict__ inv = static_cast<const F *>(a.inv);
    const int task = task_base + blockIdx.x;
    const int c0 = a.task_chunk_ptr[task], c1 = a.task_chunk_ptr[task + 1];
    const int t = threadIdx.x;
    double dacc = 0.0;
    for (int q = 0; q < c1 - c0; ++q) {
        const Chunk ch = a.chunks[FWD ? c0 + q : c1 - 1 - q];
        const int nr = ch.nrows;
        const bool active = t < nr;
        const int i = ch.row0 + t;
        F s = F(0), dinv = F(0);
        uint32_t m = 0;
        if (active) {
            s = static_cast<F>(in[i]);
            m = a.meta[i];
            dinv = inv[i];
        }
        const int ne = m & 0xffffu, ni = (m >> 16) & 0xffu, lev = m >> 24;
        const F *v = sval + ch.off + t;
        const int *cj = a.scol + ch.off + t;
        // terms already final before this chunk: all lanes at once
        for (int k = 0; k < ne; ++k) s -= v[k * nr] * static_cast<F>(out[cj[k * nr]]);
        // in-chunk terms, level by level
        for (int L = 0; L < ch.depth; ++L) {
            if (active && lev == L) {
                for (int k = ne; k < ne + ni; ++k) s -= v[k * nr] * ys[cj[k * nr] - ch.row0];
                ys[t] = s * dinv;
            }
            __syncthreads();
        }
        if (active) {
            const F yv = ys[t];
            out[i] = static_cast<TOut>(yv);
            if (rdot) dacc += rdot[i] * static_cast<double>(yv);
        }
        // later chunks of this task read this chunk's results from memory
        if (q + 1 < c1 - c0) __syncthreads();
    }
    if (part) {
        const double tsum = wave_sum(dacc);
        if (t == 0) part[task] = tsum;
    }
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
template <typename T>
struct DevArray {
    T *p = nullptr;
    size_t count = 0;
    DevArray() = default;
    DevArray(const DevArray &) = delete;
    DevArray &operator=(const DevArray &) = delete;
    ~DevArray() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        count = 0;
    }
    int alloc(size_t c) {
        release();
        if (c == 0) c = 1;
        hipError_t e = hipMalloc(&p, c * sizeof(T));
        if (e != hipSuccess) {
            p = nullptr;
            return set_error(ICCG_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        count = c;
        return ICCG_OK;
    }
    int upload(const T *h, size_t c, hipStream_t s) {
        ICCG_CHECK(alloc(c));
        if (c) HIP_CHECK(hipMemcpyAsync(p, h, c * sizeof(T), hipMemcpyHostToDevice, s));
        return ICCG_OK;
    }
};

struct DevSweep {
    int ntasks = 0;
    long long nslots = 0;
    int max_depth = 0;
    std::vector<int> color_task_ptr;
    DevArray<int> task_chunk_ptr;
    DevArray<Chunk> chunks;
    DevArray<uint32_t> meta;
    DevArray<int> scol, ssrc;
    DevArray<double> sval64;
    DevArray<float> sval32;
};

// Per-launch HIP-event timing of an instrumented (eager) solve.
enum ProfKind : int { PK_SPMV = 0, PK_FWD = 1, PK_BWD = 2, PK_COUNT = 3 };

struct Profiler {
    std::vector<hipEvent_t> pool;
    std::vector<int> kinds;       // kind of each recorded pair
    size_t used = 0;              // events used in the current round
    double ms[PK_COUNT] = {0, 0, 0};
    long long launches[PK_COUNT] = {0, 0, 0};
    ~Profiler() {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
    hipEvent_t next() {
        if (used == pool.size()) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
    void begin(hipStream_t s) {
        hipEvent_t e = next();
        if (e) (void)hipEventRecord(e, s);
    }
    void end(hipStream_t s, int kind) {
        hipEvent_t e = next();
        if (e) (void)hipEventRecord(e, s);
        kinds.push_back(kind);
    }
    // after the stream has drained: fold the recorded pairs into the totals
    void harvest() {
        for (size_t k = 0; k < kinds.size() && 2 * k + 1 < used; ++k) {
            float t = 0.0f;
            if (hipEventElapsedTime(&t, pool[2 * k], pool[2 * k + 1]) == hipSuccess) {
                ms[kinds[k]] += t;
                launches[kinds[k]] += 1;
            }
        }
        kinds.clear();
        used = 0;
    }
};

struct iccg_ctx {
    Profiler *prof = nullptr;     // set only during iccg_profile_solve
    int n = 0, nnz = 0, nnz_lower = 0, nblocks = 0, ncolors = 0, max_block = 0;
    iccg_options opt{};
    hipStream_t user = nullptr;   // caller's stream
    hipStream_t work = nullptr;   // internal stream (graph capture needs a non-null stream)
    hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_t0 = nullptr, ev_t1 = nullptr;
    std::vector<int> h_rowptr, h_col, h_dpos;
    std::vector<double> h_val;
    DevArray<int> rowptr, col, dpos;
    DevArray<double> val, lval, lstage;
    DevSweep fwd, bwd;
    DevArray<double> inv64;
    DevArray<float> inv32;
    bool has_factor = false;
    DevArray<double> x, r, z, p, q, b, y64;
    DevArray<float> y32;
    DevArray<double> part, hist;
    DevArray<DevScalars> scal;
    DevArray<int> dint;
    DevScalars *h_scal = nullptr;   // pinned
    int spmv_lanes = 8;
    int spmv_blocks = 1, vec_blocks = 1;
    hipGraphExec_t graph = nullptr;
    int graph_iters = 0;
    double last_ms = 0.0;
    int last_iters = 0;
    int last_hist = 0;

    ~iccg_ctx() {
        if (graph) (void)hipGraphExecDestroy(graph);
        if (h_scal) (void)hipHostFree(h_scal);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
        if (ev_t0) (void)hipEventDestroy(ev_t0);
        if (ev_t1) (void)hipEventDestroy(ev_t1);
        if (work) (void)hipStreamDestroy(work);
    }

    bool fp32() const { return opt.precision == ICCG_FP32; }

    // make the internal stream wait for the caller's stream
    int enter() {
        HIP_CHECK(hipEventRecord(ev_in, user));
        HIP_CHECK(hipStreamWaitEvent(work, ev_in, 0));
        return ICCG_OK;
    }
    // make the caller's stream wait for the internal stream
    int leave() {
        HIP_CHECK(hipEventRecord(ev_out, work));
        HIP_CHECK(hipStreamWaitEvent(user, ev_out, 0));
        return ICCG_OK;
    }
};

namespace {

int grid_for(long long items, int threads, int cap) {
    long long g = (items + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return static_cast<int>(g);
}

int launch_spmv(iccg_ctx *c, int mode, const double *x, double *y, const double *b,
                const DevScalars *sc) {
    const int G = c->spmv_lanes;
    dim3 grid(c->spmv_blocks), block(kVecThreads);
    if (c->prof) c->prof->begin(c->work);
#define SPMV_CASE(GG)                                                                          \
    case GG:                                                                                   \
        if (mode == 0)                                                                         \
            hipLaunchKernelGGL((k_spmv<GG, 0>), grid, block, 0, c->work, c->n, c->rowptr.p,    \
                               c->col.p, c->val.p, x, y, b, c->part.p, sc);                    \
        else                                                                                   \
            hipLaunchKernelGGL((k_spmv<GG, 1>), grid, block, 0, c->work, c->n, c->rowptr.p,    \
                               c->col.p, c->val.p, x, y, b, c->part.p, sc);                    \
        break;
    switch (G) {
        SPMV_CASE(4)
        SPMV_CASE(8)
        SPMV_CASE(16)
        SPMV_CASE(32)
        SPMV_CASE(64)
        default: return set_error(ICCG_EINVAL, "bad SpMV lane count");
    }
#undef SPMV_CASE
    if (c->prof) c->prof->end(c->work, PK_SPMV);
    HIP_CHECK(hipGetLastError());
    return ICCG_OK;
}

SweepArgs sweep_args(const iccg_ctx *c, const DevSweep &s) {
    SweepArgs a;
    a.task_chunk_ptr = s.task_chunk_ptr.p;
    a.chunks = s.chunks.p;
    a.meta = s.meta.p;
    a.scol = s.scol.p;
    if (c->fp32()) {
        a.sval = s.sval32.p;
        a.inv = c->inv32.p;
    } else {
        a.sval = s.sval64.p;
        a.inv = c->inv64.p;
    }
    return a;
}

// y = L^{-1} r with r FP64; y is FP64 (y64) or FP32 (y32) by precision.
int launch_forward(iccg_ctx *c, const double *r, void *y, const DevScalars *sc) {
    const SweepArgs a = sweep_args(c, c->fwd);
    for (int col = 0; col < c->ncolors; ++col) {
        const int t0 = c->fwd.color_task_ptr[col], t1 = c->fwd.color_task_ptr[col + 1];
        if (t1 == t0) continue;
        if (c->prof) c->prof->begin(c->work);
        if (c->fp32())
            hipLaunchKernelGGL((k_sweep<float, true, double, float>), dim3(t1 - t0), dim3(64), 0,
                               c->work, a, t0, r, static_cast<float *>(y), nullptr, nullptr, sc);
        else
            hipLaunchKernelGGL((k_sweep<double, true, double, double>), dim3(t1 - t0), dim3(64), 0,
                               c->work, a, t0, r, static_cast<double *>(y), nullptr, nullptr, sc);
        if (c->prof) c->prof->end(c->work, PK_FWD);
    }
    HIP_CHECK(hipGetLastError());
    return ICCG_OK;
}

// z = L^{-T} y; with rdot, part[task] = sum over the task's rows of rdot_i z_i.
int launch_backward(iccg_ctx *c, const void *y, double *z, const double *rdot, double *part,
                    const DevScalars *sc) {
    const SweepArgs a = sweep_args(c, c->bwd);
    for (int col = c->ncolors - 1; col >= 0; --col) {
        const int t0 = c->bwd.color_task_ptr[col], t1 = c->bwd.color_task_ptr[col + 1];
        if (t1 == t0) continue;
        if (c->prof) c->prof->begin(c->work);
        if (c->fp32())
            hipLaunchKernelGGL((k_sweep<float, false, float, double>), dim3(t1 - t0), dim3(64), 0,
                               c->work, a, t0, static_cast<const float *>(y), z, rdot, part, sc);
        else
            hipLaunchKernelGGL((k_sweep<double, false, double, double>), dim3(t1 - t0), dim3(64),
                               0, c->work, a, t0, static_cast<const double *>(y), z, rdot, part,
                               sc);
        if (c->prof) c->prof->end(c->work, PK_BWD);
    }
    HIP_CHECK(hipGetLastError());
    return ICCG_OK;
}

void *ytmp(iccg_ctx *c) { return c->fp32() ? static_cast<void *>(c->y32.p) : c->y64.p; }

int launch_reduce(iccg_ctx *c, int np, int op, double *out) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kVecThreads), 0, c->work, c->part.p, np,
                       c->scal.p, op, out, c->hist.p);
    HIP_CHECK(hipGetLastError());
    return ICCG_OK;
}

// One CG iteration (all kernels return at once after the stopping test passed).
int enqueue_iteration(iccg_ctx *c) {
    DevScalars *sc = c->scal.p;
    ICCG_CHECK(launch_spmv(c, 0, c->p.p, c->q.p, nullptr, sc));
    ICCG_CHECK(launch_reduce(c, c->spmv_blocks, OP_ALPHA, nullptr));
    hipLaunchKernelGGL(k_update_xr, dim3(c->vec_blocks), dim3(kVecThreads), 0, c->work, c->n,
                       c->x.p, c->r.p, c->p.p, c->q.p, sc, c->part.p);
    HIP_CHECK(hipGetLastError());
    ICCG_CHECK(launch_reduce(c, c->vec_blocks, OP_RR, nullptr));
    ICCG_CHECK(launch_forward(c, c->r.p, ytmp(c), sc));
    ICCG_CHECK(launch_backward(c, ytmp(c), c->z.p, c->r.p, c->part.p, sc));
    ICCG_CHECK(launch_reduce(c, c->bwd.ntasks, OP_BETA, nullptr));
    hipLaunchKernelGGL(k_update_p, dim3(c->vec_blocks), dim3(kVecThreads), 0, c->work, c->n,
                       c->p.p, c->z.p, sc);
    HIP_CHECK(hipGetLastError());
    return ICCG_OK;
}

int enqueue_batch(iccg_ctx *c, int iters) {
    for (int k = 0; k < iters; ++k) ICCG_CHECK(enqueue_iteration(c));
    return ICCG_OK;
}

int run_batch(iccg_ctx *c, int iters) {
    if (!c->opt.use_graph) return enqueue_batch(c, iters);
    if (!c->graph || c->graph_iters != iters) {
        if (c->graph) {
            HIP_CHECK(hipGraphExecDestroy(c->graph));
            c->graph = nullptr;
        }
        HIP_CHECK(hipStreamBeginCapture(c->work, hipStreamCaptureModeThreadLocal));
        int st = enqueue_batch(c, iters);
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
    d.color_task_ptr = plan.color_task_ptr;
    ICCG_CHECK(d.task_chunk_ptr.upload(plan.task_chunk_ptr.data(), plan.task_chunk_ptr.size(), c->work));
    ICCG_CHECK(d.chunks.upload(plan.chunks.data(), plan.chunks.size(), c->work));
    ICCG_CHECK(d.meta.upload(plan.meta.data(), plan.meta.size(), c->work));
    ICCG_CHECK(d.scol.upload(plan.slot_col.data(), plan.slot_col.size(), c->work));
    ICCG_CHECK(d.ssrc.upload(plan.slot_src.data(), plan.slot_src.size(), c->work));
    return ICCG_OK;
}

// Host-only checks and schedule construction (no HIP call).
struct HostSetup {
    std::vector<int> dpos, tpos;
    SweepPlan fwd, bwd;
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
    return ICCG_OK;
}

int upload_setup(iccg_ctx *c, int n, const int *rowptr, const int *col, const double *val,
                 int nblocks, int ncolors, const HostSetup &hs) {
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
    ICCG_CHECK(upload_sweep(c, hs.fwd, c->fwd));
    ICCG_CHECK(upload_sweep(c, hs.bwd, c->bwd));
    ICCG_CHECK(c->lval.alloc(nnz));
    if (c->fp32()) {
        ICCG_CHECK(c->inv32.alloc(n));
        ICCG_CHECK(c->y32.alloc(n));
    } else {
        ICCG_CHECK(c->inv64.alloc(n));
    }
    ICCG_CHECK(c->y64.alloc(n));
    for (DevArray<double> *v : {&c->x, &c->r, &c->z, &c->p, &c->q, &c->b}) ICCG_CHECK(v->alloc(n));

    // SpMV: lanes per row = power of two near the mean row length
    const double mean = static_cast<double>(nnz) / n;
    int G = 4;
    while (G < 64 && G < mean * 0.75) G *= 2;
    c->spmv_lanes = G;
    const int rows_per_block = kVecThreads / G;
    c->spmv_blocks = grid_for(n, rows_per_block, 8192);
    c->vec_blocks = grid_for(n, kVecThreads, kMaxVecBlocks);
    const int np = std::max({c->spmv_blocks, c->vec_blocks, c->bwd.ntasks, c->fwd.ntasks, 1});
    ICCG_CHECK(c->part.alloc(np));
    ICCG_CHECK(c->scal.alloc(1));
    ICCG_CHECK(c->dint.alloc(1));
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
    HIP_CHECK(hipStreamSynchronize(c->work));
    return ICCG_OK;
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
    ICCG_CHECK(launch_spmv(c, 1, c->x.p, c->r.p, c->b.p, nullptr));
    ICCG_CHECK(launch_reduce(c, c->spmv_blocks, OP_INIT_RR, nullptr));
    // z = M^{-1} r, rho = (r, z), p = z
    ICCG_CHECK(launch_forward(c, c->r.p, ytmp(c), c->scal.p));
    ICCG_CHECK(launch_backward(c, ytmp(c), c->z.p, c->r.p, c->part.p, c->scal.p));
    ICCG_CHECK(launch_reduce(c, c->bwd.ntasks, OP_RHO, nullptr));
    hipLaunchKernelGGL(k_copy, dim3(c->vec_blocks), dim3(kVecThreads), 0, s, n, c->p.p, c->z.p, c->scal.p);
    HIP_CHECK(hipGetLastError());
    ICCG_CHECK(read_scalars(c));
    const int batch = std::max(1, c->opt.check_every);
    while (c->h_scal->done == DONE_RUNNING) {
        if (c->prof) {
            // instrumented: one eager iteration at a time, events harvested
            ICCG_CHECK(enqueue_iteration(c));
            ICCG_CHECK(read_scalars(c));
            c->prof->harvest();
        } else {
            ICCG_CHECK(run_batch(c, batch));
            ICCG_CHECK(read_scalars(c));
        }
    }
    // true residual
    ICCG_CHECK(launch_spmv(c, 1, c->x.p, c->q.p, c->b.p, nullptr));
    ICCG_CHECK(launch_reduce(c, c->spmv_blocks, OP_TRUE, nullptr));
    HIP_CHECK(hipMemcpyAsync(x, c->x.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    HIP_CHECK(hipEventRecord(c->ev_t1, s));
    ICCG_CHECK(read_scalars(c));
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
        HostSetup hs;
        ICCG_CHECK(validate(n, rowptr, col, val, nblocks, block_ptr, ncolors, color_ptr,
                            c->opt.pack_rows, hs));
        c->user = static_cast<hipStream_t>(c->opt.stream);
        HIP_CHECK(hipStreamCreateWithFlags(&c->work, hipStreamNonBlocking));
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
        std::vector<double> lv;
        const int row = ic0_host(c->n, c->h_rowptr.data(), c->h_col.data(), c->h_val.data(),
                                 c->h_dpos.data(), lv);
        if (row >= 0) {
            c->has_factor = false;
            if (breakdown_row) *breakdown_row = row;
            return set_error(ICCG_EBREAKDOWN, "IC(0) pivot not positive at row " + std::to_string(row));
        }
        HIP_CHECK(hipMemcpyAsync(c->lval.p, lv.data(), sizeof(double) * lv.size(), hipMemcpyHostToDevice, c->work));
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
        ICCG_CHECK(launch_forward(c, r, ytmp(c), nullptr));
        return launch_backward(c, ytmp(c), z, nullptr, nullptr, nullptr);
    });
}

int ic_forward(iccg_ctx *c, const double *r, double *y) {
    return entry(c, [&]() -> int {
        if (!r || !y) return set_error(ICCG_EINVAL, "null vector");
        if (!c->has_factor) return set_error(ICCG_ESTATE, "no factor");
        if (c->fp32()) {
            ICCG_CHECK(launch_forward(c, r, c->y32.p, nullptr));
            hipLaunchKernelGGL((k_convert<double, float>), dim3(c->vec_blocks), dim3(kVecThreads), 0,
                               c->work, c->n, y, c->y32.p);
            HIP_CHECK(hipGetLastError());
            return ICCG_OK;
        }
        if (r == y) return set_error(ICCG_EINVAL, "r and y must not alias");
        return launch_forward(c, r, y, nullptr);
    });
}

int ic_backward(iccg_ctx *c, const double *y, double *z) {
    return entry(c, [&]() -> int {
        if (!y || !z) return set_error(ICCG_EINVAL, "null vector");
        if (y == z) return set_error(ICCG_EINVAL, "y and z must not alias");
        if (!c->has_factor) return set_error(ICCG_ESTATE, "no factor");
        if (c->fp32()) {
            hipLaunchKernelGGL((k_convert<float, double>), dim3(c->vec_blocks), dim3(kVecThreads), 0,
                               c->work, c->n, c->y32.p, y);
            HIP_CHECK(hipGetLastError());
            return launch_backward(c, c->y32.p, z, nullptr, nullptr, nullptr);
        }
        return launch_backward(c, y, z, nullptr, nullptr, nullptr);
    });
}

int iccg_spmv(iccg_ctx *c, const double *p, double *q, double *pq_host) {
    return entry(c, [&]() -> int {
        if (!p || !q || p == q) return set_error(ICCG_EINVAL, "need distinct p and q");
        ICCG_CHECK(launch_spmv(c, 0, p, q, nullptr, nullptr));
        if (pq_host) {
            ICCG_CHECK(launch_reduce(c, c->spmv_blocks, OP_STORE, c->b.p));
            HIP_CHECK(hipMemcpyAsync(pq_host, c->b.p, sizeof(double), hipMemcpyDeviceToHost, c->work));
            HIP_CHECK(hipStreamSynchronize(c->work));
        }
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

int iccg_solve(iccg_ctx *c, const double *b, double *x, double tol, int maxit, int *iters,
               double *relres, double *relres_true) {
    return entry(c, [&]() -> int { return solve_impl(c, b, x, tol, maxit, iters, relres, relres_true); });
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
    return ICCG_OK;
}

}  // extern "C"
