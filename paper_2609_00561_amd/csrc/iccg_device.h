// Device-side declarations shared by the HIP sources of libiccg.so: error
// macros, device scalars of a CG solve, device arrays and the context.
#pragma once

#include <hip/hip_runtime.h>

#include "iccg_internal.h"

#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

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

// Wide tasks of one sweep direction (WidePlan on the device).
struct DevWide {
    int nwide = 0;
    long long nslots = 0;
    std::vector<int> color_ptr;      // wide tasks of each color
    DevArray<int> task, piece_ptr;
    DevArray<WidePiece> pieces;
    DevArray<Chunk> subs;
    DevArray<uint32_t> wmeta;
    DevArray<int> wlev;
    DevArray<int> scol, ssrc;
    DevArray<double> sval64;
    DevArray<float> sval32;
};

struct DevSweep {
    int ntasks = 0;
    long long nslots = 0;
    int max_depth = 0;
    int max_width = 0;
    int kmax = 4;                      // register slots per row (widest row of the sweep)
    std::vector<int> color_kmax;       // per color: the tier of its widest row
    std::vector<int> color_task_ptr;
    DevArray<TaskRec> tasks;
    DevArray<Chunk> chunks;
    DevArray<uint32_t> meta;
    DevArray<int> scol, ssrc;
    DevArray<double> sval64;
    DevArray<float> sval32;
    // single-launch sweep: sweep number, per-task flags, dependency lists
    DevArray<int> epoch;            // sweep number, bumped before every launch
    DevArray<int> flag_loc, flag_rem, deps, wg_task;   // dependency ranges sit in the task records
    long long ndeps = 0;
    long long remote_tasks = 0, exported_rows = 0;
    DevWide wide;                   // per-color launches only
};

// Per-launch HIP-event timing of an instrumented (eager) solve.
enum ProfKind : int { PK_SPMV = 0, PK_FWD = 1, PK_BWD = 2, PK_COUNT = 3 };

// Device time per kind of kernel: one event pair brackets each run of
// back-to-back launches of one kind (all colors of a sweep, one SpMV), so the
// bracket adds no gap between the kernels it times.
struct Profiler {
    std::vector<hipEvent_t> pool;
    std::vector<int> kinds;       // kind of each recorded pair
    std::vector<int> counts;      // launches inside each recorded pair
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
    void end(hipStream_t s, int kind, int count = 1) {
        hipEvent_t e = next();
        if (e) (void)hipEventRecord(e, s);
        kinds.push_back(kind);
        counts.push_back(count);
    }
    // after the stream has drained: fold the recorded pairs into the totals
    void harvest() {
        for (size_t k = 0; k < kinds.size() && 2 * k + 1 < used; ++k) {
            float t = 0.0f;
            if (hipEventElapsedTime(&t, pool[2 * k], pool[2 * k + 1]) == hipSuccess) {
                ms[kinds[k]] += t;
                launches[kinds[k]] += counts[k];
            }
        }
        kinds.clear();
        counts.clear();
        used = 0;
    }
};

struct LearnedFeatures;
void destroy_learned_features(LearnedFeatures *f);

struct iccg_ctx {
    Profiler *prof = nullptr;     // set only during iccg_profile_solve
    int n = 0, nnz = 0, nnz_lower = 0, nblocks = 0, ncolors = 0, max_block = 0;
    double stats6[6] = {0, 0, 0, 0, 0, 0};   // iccg_block_stats of the ordering
    iccg_options opt{};
    hipStream_t user = nullptr;   // caller's stream
    hipStream_t work = nullptr;   // internal stream (graph capture needs a non-null stream)
    hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_t0 = nullptr, ev_t1 = nullptr;
    std::vector<int> h_rowptr, h_col, h_dpos;
    std::vector<double> h_val;
    DevArray<int> rowptr, col, dpos, tpos;
    DevArray<double> val, lval, lstage;
    DevArray<double> lval0;        // the IC(0) factor (input of the learned form)
    bool has_ic0 = false;
    LearnedFeatures *feat = nullptr;   // learned-form features of A', built on first use
    DevSweep fwd, bwd;
    DevArray<double> inv64;
    DevArray<float> inv32;
    bool has_factor = false;
    DevArray<double> x, r, z, p, q, b, y64;
    DevArray<float> y32;
    DevArray<double> part, part_rr, hist;   // partial sums; part_rr: ||r||^2 per forward task
    DevArray<DevScalars> scal;
    DevArray<int> dint;
    DevArray<int> sweep_err;       // set by a sweep wait that exceeded its spin limit
    DevScalars *h_scal = nullptr;   // pinned
    // blocks of right-hand sides (iccg_solve_multi): k columns of n, ld = n
    int mk = 0;                     // columns the buffers below hold
    DevArray<double> mx, mr, mz, mp, mq, mb, my64;
    DevArray<float> my32;
    DevArray<double> mpart, mpart_rr, mhist;
    DevArray<DevScalars> mscal;
    DevScalars *h_mscal = nullptr;  // pinned, kMaxCols of them
    int mhist_cap = 0;
    hipGraphExec_t mgraph = nullptr;
    int mgraph_iters = 0, mgraph_k = 0;
    int h_err = 0;
    int nslices = 0;                // sliced ELL copy of A' for the SpMV
    int sell_wmax = 8;              // register slots per row in k_spmv
    DevArray<int4> sell_rec;        // per launch position: slice, first slot, width
    DevArray<int> sell_order, sell_col;
    DevArray<double> sell_val;
    int spmv_blocks = 1, vec_blocks = 1;
    hipGraphExec_t graph = nullptr;
    int graph_iters = 0;
    long long flow_sweeps = 0;    // single-launch sweeps since the flags were last cleared
    int num_cu = 0;                 // compute units of the device
    int device = 0;                 // HIP device current at iccg_setup
    int last_resident = 0;          // workgroups of the last single-launch sweep
    int flow_tail = 0;              // hybrid sweeps: first color of the dataflow part
    std::unordered_map<const void *, int> resident;   // resident workgroups per CU, per kernel
    double last_ms = 0.0;
    int last_iters = 0;
    int last_hist = 0;

    ~iccg_ctx() {
        if (feat) destroy_learned_features(feat);
        if (graph) (void)hipGraphExecDestroy(graph);
        if (mgraph) (void)hipGraphExecDestroy(mgraph);
        if (h_scal) (void)hipHostFree(h_scal);
        if (h_mscal) (void)hipHostFree(h_mscal);
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

