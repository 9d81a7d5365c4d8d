// Learned IC(0) correction: a small message-passing network predicts
// corrections to the IC(0) factor values on the same sparsity pattern, so the
// substitution sweeps stay as they are.  The paper has no learned component;
// this is the added learned-factor form.  Training (FP32) and inference (FP32
// or BF16 storage with FP32 accumulation) run in the kernels below.
//
// Network (scaled space: s_i = 1/sqrt(a'_ii), A~ = S A' S, L~0 = S L0):
//   node features x_i = [L~0_ii, sum_{j!=i} |A~_ij|, deg_i/26]
//   edge features f_k = [A~_ij, [j<i], [j==i], L~0 at the lower position of (i,j)]
//   3 layers of width 32:  p_k = W_m [h_j; f_k] + b_m  (off-diagonal k = (i,j))
//                          h'_i = relu(W_s h_i + b + sum_k relu(p_k))
//   readout on lower entries k = (i,j), j <= i:
//                          delta_k = w_o . relu(W_r [h_i; h_j; f_k] + b_r) + b_o
//   L~ = L~0 + 0.1 delta;   factor of A':  L_k = L0_k + 0.1 delta_k / s_i
//   loss = mean over probes z of ||L~ L~^T z - A~ z||^2 / ||A~ z||^2
// Parameter layout: per layer (W_s[32][d], b[32], W_m[32][d+4], b_m[32]),
// d = 3, 32, 32; then W_r[32][68], b_r[32], w_o[32], b_o.
#include "iccg_device.h"

#include <algorithm>
#include <cmath>
#include <memory>

namespace {

constexpr int HID = 32;
constexpr int NFEAT = 3;
constexpr int EFEAT = 4;
constexpr int NLAYER = 3;
constexpr int RIN = 2 * HID + EFEAT;   // readout input width
constexpr float kCorr = 0.1f;
constexpr int kGemmWG = 256;
constexpr int kGemmTile = 64;
constexpr int kGemmGroups = 128;

struct Layout {
    int din[NLAYER];
    int ws[NLAYER], b[NLAYER], wm[NLAYER], bm[NLAYER];
    int wr, br, wo, bo, total;
};

constexpr Layout make_layout() {
    Layout L{};
    int k = 0;
    for (int l = 0; l < NLAYER; ++l) {
        const int d = (l == 0) ? NFEAT : HID;
        L.din[l] = d;
        L.ws[l] = k; k += HID * d;
        L.b[l] = k; k += HID;
        L.wm[l] = k; k += HID * (d + EFEAT);
        L.bm[l] = k; k += HID;
    }
    L.wr = k; k += HID * RIN;
    L.br = k; k += HID;
    L.wo = k; k += HID;
    L.bo = k; k += 1;
    L.total = k;
    return L;
}

constexpr Layout kL = make_layout();

// ---------------------------------------------------------------------------
// storage types: FP32, or BF16 (round to nearest even) with FP32 arithmetic
// ---------------------------------------------------------------------------
struct bf16 {
    uint16_t bits;
};

__device__ __forceinline__ float to_f(float v) { return v; }
__device__ __forceinline__ float to_f(bf16 v) { return __uint_as_float(static_cast<uint32_t>(v.bits) << 16); }
template <typename T> __device__ __forceinline__ T from_f(float v);
template <> __device__ __forceinline__ float from_f<float>(float v) { return v; }
template <> __device__ __forceinline__ bf16 from_f<bf16>(float v) {
    const uint32_t u = __float_as_uint(v);
    bf16 r;
    r.bits = static_cast<uint16_t>((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
    return r;
}

__global__ void k_round_bf16(int count, const float *__restrict__ src, float *__restrict__ dst) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        dst[i] = to_f(from_f<bf16>(src[i]));
}

// ---------------------------------------------------------------------------
// features
// ---------------------------------------------------------------------------
__global__ void k_feat_scale(int n, const int *__restrict__ dpos, const double *__restrict__ val,
                             double *__restrict__ s) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        s[i] = 1.0 / sqrt(val[dpos[i]]);
}

__global__ void k_feat(int n, const int *__restrict__ rowptr, const int *__restrict__ col,
                       const int *__restrict__ tpos, const int *__restrict__ dpos,
                       const double *__restrict__ val, const double *__restrict__ lval0,
                       const double *__restrict__ s, float *__restrict__ at,
                       float *__restrict__ l0t, float4 *__restrict__ f,
                       float *__restrict__ x) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double si = s[i];
        double absum = 0.0;
        int deg = 0;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            const int j = col[k];
            const double a = val[k] * si * s[j];
            at[k] = static_cast<float>(a);
            const double lt_here = (j <= i) ? lval0[k] * si : 0.0;
            l0t[k] = static_cast<float>(lt_here);
            const double lt_low = (j <= i) ? lt_here : lval0[tpos[k]] * s[j];
            f[k] = make_float4(static_cast<float>(a), j < i ? 1.0f : 0.0f, j == i ? 1.0f : 0.0f,
                               static_cast<float>(lt_low));
            if (j != i) {
                absum += fabs(a);
                ++deg;
            }
        }
        x[i * NFEAT + 0] = static_cast<float>(lval0[dpos[i]] * si);
        x[i * NFEAT + 1] = static_cast<float>(absum);
        x[i * NFEAT + 2] = static_cast<float>(deg / 26.0);
    }
}

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
// One 32-lane group per node, one lane per output channel.
template <int DIN, typename T, bool SAVE>
__global__ __launch_bounds__(256) void k_layer_fwd(int n, const int *__restrict__ rowptr,
                                                   const int *__restrict__ col,
                                                   const float4 *__restrict__ f,
                                                   const T *__restrict__ hin,
                                                   const float *__restrict__ W, int off_ws,
                                                   int off_b, int off_wm, int off_bm,
                                                   T *__restrict__ hout, float *__restrict__ apre,
                                                   float *__restrict__ P) {
    __shared__ float ws[HID * DIN], wm[HID * (DIN + EFEAT)], bb[HID], bm[HID];
    for (int t = threadIdx.x; t < HID * DIN; t += 256) ws[t] = W[off_ws + t];
    for (int t = threadIdx.x; t < HID * (DIN + EFEAT); t += 256) wm[t] = W[off_wm + t];
    if (threadIdx.x < HID) {
        bb[threadIdx.x] = W[off_b + threadIdx.x];
        bm[threadIdx.x] = W[off_bm + threadIdx.x];
    }
    __syncthreads();
    const int c = threadIdx.x & 31;
    const int i = blockIdx.x * 8 + (threadIdx.x >> 5);
    if (i >= n) return;
    float acc = bb[c];
    for (int k = 0; k < DIN; ++k) acc += ws[c * DIN + k] * to_f(hin[i * DIN + k]);
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
        const int j = col[k];
        if (j == i) continue;
        float p = bm[c];
        for (int m = 0; m < DIN; ++m) p += wm[c * (DIN + EFEAT) + m] * to_f(hin[j * DIN + m]);
        const float4 fk = f[k];
        const float *wr = wm + c * (DIN + EFEAT) + DIN;
        p += wr[0] * fk.x + wr[1] * fk.y + wr[2] * fk.z + wr[3] * fk.w;
        if (SAVE) P[static_cast<size_t>(k) * HID + c] = p;
        acc += fmaxf(p, 0.0f);
    }
    if (SAVE) apre[i * HID + c] = acc;
    hout[i * HID + c] = from_f<T>(fmaxf(acc, 0.0f));
}

// Readout on lower entries; one 32-lane group per entry.  Writes delta (and
// the pre-activations when SAVE).
template <typename T, bool SAVE>
__global__ __launch_bounds__(256) void k_readout_fwd(int nl, const int *__restrict__ lowpos,
                                                     const int *__restrict__ lowrow,
                                                     const int *__restrict__ col,
                                                     const float4 *__restrict__ f,
                                                     const T *__restrict__ h,
                                                     const float *__restrict__ W,
                                                     float *__restrict__ delta,
                                                     float *__restrict__ Q) {
    __shared__ float wr[HID * RIN], br[HID], wo[HID];
    for (int t = threadIdx.x; t < HID * RIN; t += 256) wr[t] = W[kL.wr + t];
    if (threadIdx.x < HID) {
        br[threadIdx.x] = W[kL.br + threadIdx.x];
        wo[threadIdx.x] = W[kL.wo + threadIdx.x];
    }
    __syncthreads();
    const float bo = W[kL.bo];
    const int c = threadIdx.x & 31;
    const int e = blockIdx.x * 8 + (threadIdx.x >> 5);
    float d = 0.0f;
    if (e < nl) {
        const int k = lowpos[e], i = lowrow[e], j = col[k];
        float q = br[c];
        const float *w = wr + c * RIN;
        for (int m = 0; m < HID; ++m) q += w[m] * to_f(h[i * HID + m]);
        for (int m = 0; m < HID; ++m) q += w[HID + m] * to_f(h[j * HID + m]);
        const float4 fk = f[k];
        q += w[2 * HID] * fk.x + w[2 * HID + 1] * fk.y + w[2 * HID + 2] * fk.z + w[2 * HID + 3] * fk.w;
        if (SAVE) Q[static_cast<size_t>(e) * HID + c] = q;
        d = wo[c] * fmaxf(q, 0.0f);
    }
    for (int o = 16; o > 0; o >>= 1) d += __shfl_xor(d, o, 32);
    if (e < nl && c == 0) delta[e] = d + bo;
}

// L~ at A's positions (lower only) in FP32 for the loss: L~0 + 0.1 delta.
__global__ void k_assemble_lt(int nl, const int *__restrict__ lowpos, const float *__restrict__ l0t,
                              const float *__restrict__ delta, float *__restrict__ lt) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nl; e += gridDim.x * blockDim.x) {
        const int k = lowpos[e];
        lt[k] = l0t[k] + kCorr * delta[e];
    }
}

// factor of A' in FP64: L0 + 0.1 delta / s_i on the lower positions, 0 above
__global__ void k_factor_out(int n, const int *__restrict__ rowptr, const int *__restrict__ col,
                             const int *__restrict__ lowidx, const double *__restrict__ lval0,
                             const double *__restrict__ s, const float *__restrict__ delta,
                             double *__restrict__ out) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
            out[k] = (col[k] <= i)
                         ? lval0[k] + static_cast<double>(kCorr * delta[lowidx[k]]) / s[i]
                         : 0.0;
}

// ---------------------------------------------------------------------------
// probe loss (FP64 vectors, FP32 factor values); P probes stored [P][n]
// ---------------------------------------------------------------------------
// out = A~ z
__global__ void k_probe_sym(int n, int P, const int *__restrict__ rowptr, const int *__restrict__ col,
                            const float *__restrict__ at, const double *__restrict__ Z,
                            double *__restrict__ out) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n * P; t += gridDim.x * blockDim.x) {
        const int p = t / n, i = t - p * n;
        const double *z = Z + static_cast<size_t>(p) * n;
        double s = 0.0;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) s += static_cast<double>(at[k]) * z[col[k]];
        out[t] = s;
    }
}

// out = L~^T v: row i sums L~_ji v_j over j >= i (the transposed lower entry)
__global__ void k_probe_lt(int n, int P, const int *__restrict__ rowptr, const int *__restrict__ col,
                           const int *__restrict__ tpos, const float *__restrict__ lt,
                           const double *__restrict__ V, double *__restrict__ out) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n * P; t += gridDim.x * blockDim.x) {
        const int p = t / n, i = t - p * n;
        const double *v = V + static_cast<size_t>(p) * n;
        double s = 0.0;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
            if (col[k] >= i) s += static_cast<double>(lt[tpos[k]]) * v[col[k]];
        out[t] = s;
    }
}

// out = L~ v - T
__global__ void k_probe_l_minus(int n, int P, const int *__restrict__ rowptr,
                                const int *__restrict__ col, const float *__restrict__ lt,
                                const double *__restrict__ V, const double *__restrict__ T,
                                double *__restrict__ out) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n * P; t += gridDim.x * blockDim.x) {
        const int p = t / n, i = t - p * n;
        const double *v = V + static_cast<size_t>(p) * n;
        double s = 0.0;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
            if (col[k] <= i) s += static_cast<double>(lt[k]) * v[col[k]];
        out[t] = s - T[t];
    }
}

// per probe: partial sums of ||E||^2 and ||T||^2 per workgroup (256 threads)
__global__ __launch_bounds__(256) void k_probe_norms(int n, const double *__restrict__ E,
                                                     const double *__restrict__ T,
                                                     double *__restrict__ part) {
    const int p = blockIdx.y;
    const double *e = E + static_cast<size_t>(p) * n, *t = T + static_cast<size_t>(p) * n;
    double a = 0.0, b = 0.0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        a += e[i] * e[i];
        b += t[i] * t[i];
    }
    __shared__ double ra[4], rb[4];
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        ra[threadIdx.x >> 6] = a;
        rb[threadIdx.x >> 6] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[(p * gridDim.x + blockIdx.x) * 2 + 0] = ra[0] + ra[1] + ra[2] + ra[3];
        part[(p * gridDim.x + blockIdx.x) * 2 + 1] = rb[0] + rb[1] + rb[2] + rb[3];
    }
}

// loss = mean_p ee_p / tt_p; coef[p] = 2 / (P tt_p)
__global__ void k_probe_loss(int P, int groups, const double *__restrict__ part,
                             double *__restrict__ coef, double *__restrict__ loss) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double total = 0.0;
    for (int p = 0; p < P; ++p) {
        double ee = 0.0, tt = 0.0;
        for (int g = 0; g < groups; ++g) {
            ee += part[(p * groups + g) * 2 + 0];
            tt += part[(p * groups + g) * 2 + 1];
        }
        total += ee / tt;
        coef[p] = 2.0 / (P * tt);
    }
    loss[0] = total / P;
}

// dL/dL~ on the lower entries: sum_p coef_p (E_p[i] W_p[j] + Z_p[i] GE_p[j])
__global__ void k_grad_lt(int nl, int n, int P, const int *__restrict__ lowpos,
                          const int *__restrict__ lowrow, const int *__restrict__ col,
                          const double *__restrict__ coef, const double *__restrict__ E,
                          const double *__restrict__ Wv, const double *__restrict__ Z,
                          const double *__restrict__ GE, float *__restrict__ G) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nl; e += gridDim.x * blockDim.x) {
        const int i = lowrow[e], j = col[lowpos[e]];
        double g = 0.0;
        for (int p = 0; p < P; ++p) {
            const size_t o = static_cast<size_t>(p) * n;
            g += coef[p] * (E[o + i] * Wv[o + j] + Z[o + i] * GE[o + j]);
        }
        G[e] = static_cast<float>(g);
    }
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------
// readout: DQ[e][c] = 0.1 G[e] w_o[c] [q > 0];  DD[e] = 0.1 G[e]
__global__ void k_readout_bwd(int nl, const float *__restrict__ G, const float *__restrict__ Q,
                              const float *__restrict__ W, float *__restrict__ DQ,
                              float *__restrict__ DD) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nl * HID; t += gridDim.x * blockDim.x) {
        const int e = t / HID, c = t - e * HID;
        const float dd = kCorr * G[e];
        DQ[t] = (Q[t] > 0.0f) ? dd * W[kL.wo + c] : 0.0f;
        if (c == 0) DD[e] = dd;
    }
}

// dH[i][c'] from the readout: sum over lower entries with row i of
// W_r[:, c']^T DQ plus over lower entries with column i of W_r[:, 32+c']^T DQ
__global__ __launch_bounds__(256) void k_readout_bwd_h(int n, const int *__restrict__ rowptr,
                                                       const int *__restrict__ col,
                                                       const int *__restrict__ tpos,
                                                       const int *__restrict__ lowidx,
                                                       const float *__restrict__ W,
                                                       const float *__restrict__ DQ,
                                                       float *__restrict__ dH) {
    __shared__ float wr[HID * RIN];
    for (int t = threadIdx.x; t < HID * RIN; t += 256) wr[t] = W[kL.wr + t];
    __syncthreads();
    const int cp = threadIdx.x & 31;
    const int i = blockIdx.x * 8 + (threadIdx.x >> 5);
    if (i >= n) return;
    float acc = 0.0f;
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
        const int j = col[k];
        if (j <= i) {   // (i, j) lower: node i in the first slot
            const float *dq = DQ + static_cast<size_t>(lowidx[k]) * HID;
            for (int c = 0; c < HID; ++c) acc += wr[c * RIN + cp] * dq[c];
        }
        if (j >= i) {   // (j, i) lower: node i in the second slot
            const float *dq = DQ + static_cast<size_t>(lowidx[tpos[k]]) * HID;
            for (int c = 0; c < HID; ++c) acc += wr[c * RIN + HID + cp] * dq[c];
        }
    }
    dH[i * HID + cp] = acc;
}

// DA = dH [apre > 0]
__global__ void k_relu_bwd(int count, const float *__restrict__ dH, const float *__restrict__ apre,
                           float *__restrict__ DA) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < count; t += gridDim.x * blockDim.x)
        DA[t] = (apre[t] > 0.0f) ? dH[t] : 0.0f;
}

// DP[k][c] = DA[i][c] [P[k][c] > 0] for off-diagonal k in row i; 0 on the diagonal
__global__ void k_msg_bwd(int n, const int *__restrict__ rowptr, const int *__restrict__ col,
                          const float *__restrict__ DA, const float *__restrict__ P,
                          float *__restrict__ DP) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n * HID; t += gridDim.x * blockDim.x) {
        const int i = t / HID, c = t - i * HID;
        const float da = DA[t];
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            const size_t o = static_cast<size_t>(k) * HID + c;
            DP[o] = (col[k] != i && P[o] > 0.0f) ? da : 0.0f;
        }
    }
}

// dHin[i][c'] = sum_c W_s[c][c'] DA[i][c] + sum over edges (j, i) of W_m[c][c'] DP[(j,i)][c]
template <int DIN>
__global__ __launch_bounds__(256) void k_layer_bwd_h(int n, const int *__restrict__ rowptr,
                                                     const int *__restrict__ col,
                                                     const int *__restrict__ tpos,
                                                     const float *__restrict__ W, int off_ws,
                                                     int off_wm, const float *__restrict__ DA,
                                                     const float *__restrict__ DP,
                                                     float *__restrict__ dHin) {
    __shared__ float ws[HID * DIN], wm[HID * (DIN + EFEAT)];
    for (int t = threadIdx.x; t < HID * DIN; t += 256) ws[t] = W[off_ws + t];
    for (int t = threadIdx.x; t < HID * (DIN + EFEAT); t += 256) wm[t] = W[off_wm + t];
    __syncthreads();
    const int cp = threadIdx.x & 31;
    const int i = blockIdx.x * 8 + (threadIdx.x >> 5);
    if (i >= n || cp >= DIN) return;
    float acc = 0.0f;
    const float *da = DA + static_cast<size_t>(i) * HID;
    for (int c = 0; c < HID; ++c) acc += ws[c * DIN + cp] * da[c];
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
        if (col[k] == i) continue;
        const float *dp = DP + static_cast<size_t>(tpos[k]) * HID;
        for (int c = 0; c < HID; ++c) acc += wm[c * (DIN + EFEAT) + cp] * dp[c];
    }
    dHin[i * DIN + cp] = acc;
}

// ---------------------------------------------------------------------------
// weight gradients: C[M][N] = sum_r A[r][m] B(r)[n], deterministic two pass.
// B rows are formed on the fly by a row builder (gathers of h and features,
// with a trailing 1 that yields the bias gradient).
// ---------------------------------------------------------------------------
struct RowHin {      // [h_i ; 1], rows = nodes
    const float *h;
    int d;
    __device__ float operator()(int r, int m) const { return m < d ? h[r * d + m] : 1.0f; }
};
struct RowMsg {      // [h_col(k) ; f_k ; 1], rows = CSR positions
    const float *h;
    const int *col;
    const float4 *f;
    int d;
    __device__ float operator()(int r, int m) const {
        if (m < d) return h[col[r] * d + m];
        if (m < d + EFEAT) {
            const float4 v = f[r];
            const int q = m - d;
            return q == 0 ? v.x : q == 1 ? v.y : q == 2 ? v.z : v.w;
        }
        return 1.0f;
    }
};
struct RowReadout {  // [h_i ; h_j ; f_k ; 1], rows = lower entries
    const float *h;
    const int *lowpos, *lowrow, *col;
    const float4 *f;
    __device__ float operator()(int r, int m) const {
        const int k = lowpos[r];
        if (m < HID) return h[lowrow[r] * HID + m];
        if (m < 2 * HID) return h[col[k] * HID + (m - HID)];
        if (m < RIN) {
            const float4 v = f[k];
            const int q = m - 2 * HID;
            return q == 0 ? v.x : q == 1 ? v.y : q == 2 ? v.z : v.w;
        }
        return 1.0f;
    }
};
struct RowU {        // [relu(q_e) ; 1], rows = lower entries
    const float *Q;
    __device__ float operator()(int r, int m) const {
        return m < HID ? fmaxf(Q[static_cast<size_t>(r) * HID + m], 0.0f) : 1.0f;
    }
};

template <int M, int N, class BR>
__global__ __launch_bounds__(kGemmWG) void k_atb(int R, const float *__restrict__ A, BR brow,
                                                 float *__restrict__ part) {
    constexpr int OUT = M * N;
    constexpr int PER = (OUT + kGemmWG - 1) / kGemmWG;
    __shared__ float As[kGemmTile][M];
    __shared__ float Bs[kGemmTile][N];
    float acc[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) acc[q] = 0.0f;
    const int chunk = ((R + gridDim.x - 1) / gridDim.x + kGemmTile - 1) / kGemmTile * kGemmTile;
    const int r0 = blockIdx.x * chunk, r1 = min(R, r0 + chunk);
    for (int t0 = r0; t0 < r1; t0 += kGemmTile) {
        for (int t = threadIdx.x; t < kGemmTile * M; t += kGemmWG) {
            const int rr = t / M, m = t - rr * M;
            As[rr][m] = (t0 + rr < r1) ? A[static_cast<size_t>(t0 + rr) * M + m] : 0.0f;
        }
        for (int t = threadIdx.x; t < kGemmTile * N; t += kGemmWG) {
            const int rr = t / N, m = t - rr * N;
            Bs[rr][m] = (t0 + rr < r1) ? brow(t0 + rr, m) : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int o = threadIdx.x + q * kGemmWG;
            if (o < OUT) {
                const int m = o / N, nn = o - m * N;
                float s = acc[q];
                for (int rr = 0; rr < kGemmTile; ++rr) s += As[rr][m] * Bs[rr][nn];
                acc[q] = s;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int o = threadIdx.x + q * kGemmWG;
        if (o < OUT) part[static_cast<size_t>(blockIdx.x) * OUT + o] = acc[q];
    }
}

// grad[off_w + m*(N-1) + n] = C[m][n] for n < N-1 (weights), grad[off_b + m] = C[m][N-1] (bias)
__global__ void k_atb_finish(int M, int N, int groups, const float *__restrict__ part,
                             float *__restrict__ grad, int off_w, int off_b) {
    const int OUT = M * N;
    for (int o = blockIdx.x * blockDim.x + threadIdx.x; o < OUT; o += gridDim.x * blockDim.x) {
        float s = 0.0f;
        for (int g = 0; g < groups; ++g) s += part[static_cast<size_t>(g) * OUT + o];
        const int m = o / N, nn = o - m * N;
        if (nn < N - 1) grad[off_w + m * (N - 1) + nn] = s;
        else grad[off_b + m] = s;
    }
}

__global__ void k_adam(int count, float *__restrict__ theta, const float *__restrict__ g,
                       float *__restrict__ m, float *__restrict__ v, float lr, float c1, float c2) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = 0.9f * m[i] + 0.1f * gi;
        const float vi = 0.999f * v[i] + 0.001f * gi * gi;
        m[i] = mi;
        v[i] = vi;
        theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
    }
}

int grid_of(long long items, int threads) {
    long long g = (items + threads - 1) / threads;
    return static_cast<int>(std::max(1LL, std::min(g, 65535LL)));
}

}  // namespace

// ---------------------------------------------------------------------------
// per-matrix features (kept in the context)
// ---------------------------------------------------------------------------
struct LearnedFeatures {
    int n = 0, nnz = 0, nl = 0;
    DevArray<double> s;
    DevArray<float> at, l0t, x;
    DevArray<float4> f;
    DevArray<int> lowpos, lowrow, lowidx;
};

void destroy_learned_features(LearnedFeatures *f) { delete f; }

static int ensure_features(iccg_ctx *c) {
    if (c->feat) return ICCG_OK;
    if (!c->has_ic0) return set_error(ICCG_ESTATE, "the learned form needs the IC(0) factor: call ic0_factor first");
    std::unique_ptr<LearnedFeatures> F(new LearnedFeatures());
    const int n = c->n, nnz = c->nnz;
    std::vector<int> lowpos, lowrow, lowidx(nnz, -1);
    for (int i = 0; i < n; ++i)
        for (int k = c->h_rowptr[i]; k < c->h_rowptr[i + 1]; ++k)
            if (c->h_col[k] <= i) {
                lowidx[k] = static_cast<int>(lowpos.size());
                lowpos.push_back(k);
                lowrow.push_back(i);
            }
    F->n = n;
    F->nnz = nnz;
    F->nl = static_cast<int>(lowpos.size());
    hipStream_t s = c->work;
    ICCG_CHECK(F->lowpos.upload(lowpos.data(), lowpos.size(), s));
    ICCG_CHECK(F->lowrow.upload(lowrow.data(), lowrow.size(), s));
    ICCG_CHECK(F->lowidx.upload(lowidx.data(), lowidx.size(), s));
    ICCG_CHECK(F->s.alloc(n));
    ICCG_CHECK(F->at.alloc(nnz));
    ICCG_CHECK(F->l0t.alloc(nnz));
    ICCG_CHECK(F->f.alloc(nnz));
    ICCG_CHECK(F->x.alloc(static_cast<size_t>(n) * NFEAT));
    hipLaunchKernelGGL(k_feat_scale, dim3(grid_of(n, 256)), dim3(256), 0, s, n, c->dpos.p, c->val.p, F->s.p);
    hipLaunchKernelGGL(k_feat, dim3(grid_of(n, 256)), dim3(256), 0, s, n, c->rowptr.p, c->col.p, c->tpos.p,
                       c->dpos.p, c->val.p, c->lval0.p, F->s.p, F->at.p, F->l0t.p, F->f.p, F->x.p);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(s));   // lowpos etc. host vectors are released on return
    c->feat = F.release();
    return ICCG_OK;
}

// ---------------------------------------------------------------------------
// network object
// ---------------------------------------------------------------------------
struct iccg_mpnn {
    hipStream_t user = nullptr, work = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    DevArray<float> theta, grad, m, v, theta_bf16;
    int step = 0;
    // work buffers, sized for the largest matrix seen
    int cap_n = 0, cap_nnz = 0, cap_nnz_train = 0, cap_nl = 0, cap_p = 0;
    DevArray<float> H[NLAYER + 1];         // H[0] = x (float), H[l] = layer outputs
    DevArray<bf16> Hb[NLAYER + 1];         // BF16 activations for inference
    DevArray<float> Apre[NLAYER], P[NLAYER];
    DevArray<float> Q, delta, lt, G, DQ, DD, dH, dH2, DA, DP, part;
    DevArray<double> T, Wv, E, GE, npart, coef, loss;
    ~iccg_mpnn() {
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
        if (work) (void)hipStreamDestroy(work);
    }
    int enter() {
        HIP_CHECK(hipEventRecord(ev_in, user));
        HIP_CHECK(hipStreamWaitEvent(work, ev_in, 0));
        return ICCG_OK;
    }
    int leave() {
        HIP_CHECK(hipEventRecord(ev_out, work));
        HIP_CHECK(hipStreamWaitEvent(user, ev_out, 0));
        return ICCG_OK;
    }
};

static int ensure_buffers(iccg_mpnn *m, int n, int nnz, int nl, int P, bool train) {
    if (n > m->cap_n) {
        for (int l = 0; l <= NLAYER; ++l) {
            ICCG_CHECK(m->H[l].alloc(static_cast<size_t>(n) * HID));
            ICCG_CHECK(m->Hb[l].alloc(static_cast<size_t>(n) * HID));
        }
        for (int l = 0; l < NLAYER; ++l) ICCG_CHECK(m->Apre[l].alloc(static_cast<size_t>(n) * HID));
        ICCG_CHECK(m->dH.alloc(static_cast<size_t>(n) * HID));
        ICCG_CHECK(m->dH2.alloc(static_cast<size_t>(n) * HID));
        ICCG_CHECK(m->DA.alloc(static_cast<size_t>(n) * HID));
        m->cap_n = n;
        m->cap_p = 0;     // probe buffers scale with n
    }
    if (nnz > m->cap_nnz) {
        ICCG_CHECK(m->lt.alloc(nnz));
        m->cap_nnz = nnz;
        m->cap_nnz_train = 0;
    }
    if (train && nnz > m->cap_nnz_train) {
        for (int l = 0; l < NLAYER; ++l) ICCG_CHECK(m->P[l].alloc(static_cast<size_t>(nnz) * HID));
        ICCG_CHECK(m->DP.alloc(static_cast<size_t>(nnz) * HID));
        m->cap_nnz_train = nnz;
    }
    if (nl > m->cap_nl) {
        ICCG_CHECK(m->Q.alloc(static_cast<size_t>(nl) * HID));
        ICCG_CHECK(m->DQ.alloc(static_cast<size_t>(nl) * HID));
        ICCG_CHECK(m->delta.alloc(nl));
        ICCG_CHECK(m->G.alloc(nl));
        ICCG_CHECK(m->DD.alloc(nl));
        m->cap_nl = nl;
    }
    if (P > m->cap_p) {
        for (DevArray<double> *a : {&m->T, &m->Wv, &m->E, &m->GE})
            ICCG_CHECK(a->alloc(static_cast<size_t>(n) * P));
        ICCG_CHECK(m->npart.alloc(static_cast<size_t>(P) * 64 * 2));
        ICCG_CHECK(m->coef.alloc(P));
        m->cap_p = P;
    }
    if (!m->loss.p) ICCG_CHECK(m->loss.alloc(1));
    if (!m->part.p) ICCG_CHECK(m->part.alloc(static_cast<size_t>(kGemmGroups) * HID * (RIN + 1)));
    return ICCG_OK;
}

// The forward is written out per precision below to keep the launch code plain.
static int forward_fp32(iccg_mpnn *m, iccg_ctx *c, bool save) {
    LearnedFeatures *F = c->feat;
    const int n = F->n, nl = F->nl;
    hipStream_t s = m->work;
    const dim3 gnode(grid_of(n, 8)), b256(256);
    const float *W = m->theta.p;
    HIP_CHECK(hipMemcpyAsync(m->H[0].p, F->x.p, sizeof(float) * n * NFEAT, hipMemcpyDeviceToDevice, s));
    for (int l = 0; l < NLAYER; ++l) {
        float *ap = save ? m->Apre[l].p : nullptr;
        float *pp = save ? m->P[l].p : nullptr;
        if (l == 0) {
            if (save)
                hipLaunchKernelGGL((k_layer_fwd<NFEAT, float, true>), gnode, b256, 0, s, n, c->rowptr.p, c->col.p,
                                   F->f.p, m->H[0].p, W, kL.ws[0], kL.b[0], kL.wm[0], kL.bm[0], m->H[1].p, ap, pp);
            else
                hipLaunchKernelGGL((k_layer_fwd<NFEAT, float, false>), gnode, b256, 0, s, n, c->rowptr.p, c->col.p,
                                   F->f.p, m->H[0].p, W, kL.ws[0], kL.b[0], kL.wm[0], kL.bm[0], m->H[1].p, ap, pp);
        } else {
            if (save)
                hipLaunchKernelGGL((k_layer_fwd<HID, float, true>), gnode, b256, 0, s, n, c->rowptr.p, c->col.p,
                                   F->f.p, m->H[l].p, W, kL.ws[l], kL.b[l], kL.wm[l], kL.bm[l], m->H[l + 1].p, ap, pp);
            else
                hipLaunchKernelGGL((k_layer_fwd<HID, float, false>), gnode, b256, 0, s, n, c->rowptr.p, c->col.p,
                                   F->f.p, m->H[l].p, W, kL.ws[l], kL.b[l], kL.wm[l], kL.bm[l], m->H[l + 1].p, ap, pp);
        }
    }
    if (save)
        hipLaunchKernelGGL((k_readout_fwd<float, true>), dim3(grid_of(nl, 8)), b256, 0, s, nl, F->lowpos.p,
                           F->lowrow.p, c->col.p, F->f.p, m->H[NLAYER].p, W, m->delta.p, m->Q.p);
    else
        hipLaunchKernelGGL((k_readout_fwd<float, false>), dim3(grid_of(nl, 8)), b256, 0, s, nl, F->lowpos.p,
                           F->lowrow.p, c->col.p, F->f.p, m->H[NLAYER].p, W, m->delta.p, m->Q.p);
    HIP_CHECK(hipGetLastError());
    return ICCG_OK;
}

__global__ void k_to_bf16(int count, const float *__restrict__ src, bf16 *__restrict__ dst) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        dst[i] = from_f<bf16>(src[i]);
}

// BF16 inference: weights rounded to BF16, activations stored in BF16, FP32 sums
static int forward_bf16(iccg_mpnn *m, iccg_ctx *c) {
    LearnedFeatures *F = c->feat;
    const int n = F->n, nl = F->nl;
    hipStream_t s = m->work;
    const dim3 gnode(grid_of(n, 8)), b256(256);
    if (!m->theta_bf16.p) ICCG_CHECK(m->theta_bf16.alloc(kL.total));
    hipLaunchKernelGGL(k_round_bf16, dim3(grid_of(kL.total, 256)), b256, 0, s, kL.total, m->theta.p, m->theta_bf16.p);
    const float *W = m->theta_bf16.p;
    hipLaunchKernelGGL(k_to_bf16, dim3(grid_of(n * NFEAT, 256)), b256, 0, s, n * NFEAT, F->x.p, m->Hb[0].p);
    hipLaunchKernelGGL((k_layer_fwd<NFEAT, bf16, false>), gnode, b256, 0, s, n, c->rowptr.p, c->col.p, F->f.p,
                       m->Hb[0].p, W, kL.ws[0], kL.b[0], kL.wm[0], kL.bm[0], m->Hb[1].p, nullptr, nullptr);
    for (int l = 1; l < NLAYER; ++l)
        hipLaunchKernelGGL((k_layer_fwd<HID, bf16, false>), gnode, b256, 0, s, n, c->rowptr.p, c->col.p, F->f.p,
                           m->Hb[l].p, W, kL.ws[l], kL.b[l], kL.wm[l], kL.bm[l], m->Hb[l + 1].p, nullptr, nullptr);
    hipLaunchKernelGGL((k_readout_fwd<bf16, false>), dim3(grid_of(nl, 8)), b256, 0, s, nl, F->lowpos.p,
                       F->lowrow.p, c->col.p, F->f.p, m->Hb[NLAYER].p, W, m->delta.p, m->Q.p);
    HIP_CHECK(hipGetLastError());
    return ICCG_OK;
}

// loss and dL/dL~ for the probes Zd [P][n] (FP64, device)
static int probe_loss(iccg_mpnn *m, iccg_ctx *c, const double *Zd, int P) {
    LearnedFeatures *F = c->feat;
    const int n = F->n, nl = F->nl, nnz = F->nnz;
    hipStream_t s = m->work;
    const dim3 b256(256);
    HIP_CHECK(hipMemsetAsync(m->lt.p, 0, sizeof(float) * nnz, s));
    hipLaunchKernelGGL(k_assemble_lt, dim3(grid_of(nl, 256)), b256, 0, s, nl, F->lowpos.p, F->l0t.p, m->delta.p, m->lt.p);
    const dim3 gv(grid_of(static_cast<long long>(n) * P, 256));
    hipLaunchKernelGGL(k_probe_sym, gv, b256, 0, s, n, P, c->rowptr.p, c->col.p, F->at.p, Zd, m->T.p);
    hipLaunchKernelGGL(k_probe_lt, gv, b256, 0, s, n, P, c->rowptr.p, c->col.p, c->tpos.p, m->lt.p, Zd, m->Wv.p);
    hipLaunchKernelGGL(k_probe_l_minus, gv, b256, 0, s, n, P, c->rowptr.p, c->col.p, m->lt.p, m->Wv.p, m->T.p, m->E.p);
    hipLaunchKernelGGL(k_probe_lt, gv, b256, 0, s, n, P, c->rowptr.p, c->col.p, c->tpos.p, m->lt.p, m->E.p, m->GE.p);
    const int groups = 64;
    hipLaunchKernelGGL(k_probe_norms, dim3(groups, P), b256, 0, s, n, m->E.p, m->T.p, m->npart.p);
    hipLaunchKernelGGL(k_probe_loss, dim3(1), dim3(64), 0, s, P, groups, m->npart.p, m->coef.p, m->loss.p);
    hipLaunchKernelGGL(k_grad_lt, dim3(grid_of(nl, 256)), b256, 0, s, nl, n, P, F->lowpos.p, F->lowrow.p, c->col.p,
                       m->coef.p, m->E.p, m->Wv.p, Zd, m->GE.p, m->G.p);
    HIP_CHECK(hipGetLastError());
    return ICCG_OK;
}

template <int M, int N, class BR>
static int weight_grad(iccg_mpnn *m, int R, const float *A, BR br, int off_w, int off_b) {
    hipStream_t s = m->work;
    hipLaunchKernelGGL((k_atb<M, N, BR>), dim3(kGemmGroups), dim3(kGemmWG), 0, s, R, A, br, m->part.p);
    hipLaunchKernelGGL(k_atb_finish, dim3(grid_of(M * N, 256)), dim3(256), 0, s, M, N, kGemmGroups, m->part.p,
                       m->grad.p, off_w, off_b);
    HIP_CHECK(hipGetLastError());
    return ICCG_OK;
}

static int backward(iccg_mpnn *m, iccg_ctx *c) {
    LearnedFeatures *F = c->feat;
    const int n = F->n, nl = F->nl, nnz = F->nnz;
    hipStream_t s = m->work;
    const dim3 b256(256), gnode(grid_of(n, 8));
    const float *W = m->theta.p;
    // readout
    hipLaunchKernelGGL(k_readout_bwd, dim3(grid_of(static_cast<long long>(nl) * HID, 256)), b256, 0, s, nl, m->G.p,
                       m->Q.p, W, m->DQ.p, m->DD.p);
    RowReadout rr{m->H[NLAYER].p, F->lowpos.p, F->lowrow.p, c->col.p, F->f.p};
    ICCG_CHECK((weight_grad<HID, RIN + 1>(m, nl, m->DQ.p, rr, kL.wr, kL.br)));
    RowU ru{m->Q.p};
    ICCG_CHECK((weight_grad<1, HID + 1>(m, nl, m->DD.p, ru, kL.wo, kL.bo)));
    hipLaunchKernelGGL(k_readout_bwd_h, gnode, b256, 0, s, n, c->rowptr.p, c->col.p, c->tpos.p, F->lowidx.p, W,
                       m->DQ.p, m->dH.p);
    // layers, last to first; dH holds d loss / d H[l+1]
    for (int l = NLAYER - 1; l >= 0; --l) {
        const int d = kL.din[l];
        hipLaunchKernelGGL(k_relu_bwd, dim3(grid_of(static_cast<long long>(n) * HID, 256)), b256, 0, s, n * HID,
                           m->dH.p, m->Apre[l].p, m->DA.p);
        hipLaunchKernelGGL(k_msg_bwd, dim3(grid_of(static_cast<long long>(n) * HID, 256)), b256, 0, s, n,
                           c->rowptr.p, c->col.p, m->DA.p, m->P[l].p, m->DP.p);
        if (d == NFEAT) {
            RowHin rh{m->H[l].p, d};
            ICCG_CHECK((weight_grad<HID, NFEAT + 1>(m, n, m->DA.p, rh, kL.ws[l], kL.b[l])));
            RowMsg rm{m->H[l].p, c->col.p, F->f.p, d};
            ICCG_CHECK((weight_grad<HID, NFEAT + EFEAT + 1>(m, nnz, m->DP.p, rm, kL.wm[l], kL.bm[l])));
        } else {
            RowHin rh{m->H[l].p, d};
            ICCG_CHECK((weight_grad<HID, HID + 1>(m, n, m->DA.p, rh, kL.ws[l], kL.b[l])));
            RowMsg rm{m->H[l].p, c->col.p, F->f.p, d};
            ICCG_CHECK((weight_grad<HID, HID + EFEAT + 1>(m, nnz, m->DP.p, rm, kL.wm[l], kL.bm[l])));
            hipLaunchKernelGGL(k_layer_bwd_h<HID>, gnode, b256, 0, s, n, c->rowptr.p, c->col.p, c->tpos.p, W,
                               kL.ws[l], kL.wm[l], m->DA.p, m->DP.p, m->dH2.p);
            std::swap(m->dH.p, m->dH2.p);
        }
    }
    HIP_CHECK(hipGetLastError());
    return ICCG_OK;
}

template <typename Fn>
static int mpnn_entry(iccg_mpnn *m, iccg_ctx *c, Fn &&body) {
    try {
        if (!m || !c) return set_error(ICCG_EINVAL, "null network or context");
        ICCG_CHECK(c->enter());
        ICCG_CHECK(m->enter());
        int st = ensure_features(c);
        if (st == ICCG_OK) {
            // the network stream waits for the context's setup work
            HIP_CHECK(hipEventRecord(c->ev_out, c->work));
            HIP_CHECK(hipStreamWaitEvent(m->work, c->ev_out, 0));
            st = body();
        }
        const int st2 = m->leave();
        HIP_CHECK(hipEventRecord(m->ev_out, m->work));
        HIP_CHECK(hipStreamWaitEvent(c->work, m->ev_out, 0));
        const int st3 = c->leave();
        return st != ICCG_OK ? st : (st2 != ICCG_OK ? st2 : st3);
    } catch (const std::bad_alloc &) {
        return set_error(ICCG_ENOMEM, "host allocation failed");
    }
}

extern "C" {

int iccg_mpnn_param_count(void) { return kL.total; }

int iccg_mpnn_create(iccg_mpnn **out, const float *params, void *stream) {
    if (!out || !params) return set_error(ICCG_EINVAL, "null argument");
    *out = nullptr;
    try {
        std::unique_ptr<iccg_mpnn> m(new iccg_mpnn());
        m->user = static_cast<hipStream_t>(stream);
        HIP_CHECK(hipStreamCreateWithFlags(&m->work, hipStreamNonBlocking));
        HIP_CHECK(hipEventCreateWithFlags(&m->ev_in, hipEventDisableTiming));
        HIP_CHECK(hipEventCreateWithFlags(&m->ev_out, hipEventDisableTiming));
        ICCG_CHECK(m->theta.upload(params, kL.total, m->work));
        ICCG_CHECK(m->grad.alloc(kL.total));
        ICCG_CHECK(m->m.alloc(kL.total));
        ICCG_CHECK(m->v.alloc(kL.total));
        HIP_CHECK(hipMemsetAsync(m->m.p, 0, sizeof(float) * kL.total, m->work));
        HIP_CHECK(hipMemsetAsync(m->v.p, 0, sizeof(float) * kL.total, m->work));
        HIP_CHECK(hipStreamSynchronize(m->work));
        *out = m.release();
        return ICCG_OK;
    } catch (const std::bad_alloc &) {
        return set_error(ICCG_ENOMEM, "host allocation failed");
    }
}

void iccg_mpnn_destroy(iccg_mpnn *m) {
    if (!m) return;
    if (m->work) (void)hipStreamSynchronize(m->work);
    delete m;
}

int iccg_mpnn_get_params(iccg_mpnn *m, float *out) {
    if (!m || !out) return set_error(ICCG_EINVAL, "null argument");
    HIP_CHECK(hipMemcpyAsync(out, m->theta.p, sizeof(float) * kL.total, hipMemcpyDeviceToHost, m->work));
    HIP_CHECK(hipStreamSynchronize(m->work));
    return ICCG_OK;
}

int iccg_mpnn_set_params(iccg_mpnn *m, const float *params) {
    if (!m || !params) return set_error(ICCG_EINVAL, "null argument");
    HIP_CHECK(hipMemcpyAsync(m->theta.p, params, sizeof(float) * kL.total, hipMemcpyHostToDevice, m->work));
    HIP_CHECK(hipMemsetAsync(m->m.p, 0, sizeof(float) * kL.total, m->work));
    HIP_CHECK(hipMemsetAsync(m->v.p, 0, sizeof(float) * kL.total, m->work));
    HIP_CHECK(hipStreamSynchronize(m->work));
    m->step = 0;
    return ICCG_OK;
}

int iccg_mpnn_loss_grad(iccg_mpnn *m, iccg_ctx *c, const double *probes, int nprobes,
                        double *loss, float *grad) {
    if (!probes || nprobes < 1) return set_error(ICCG_EINVAL, "need probes");
    return mpnn_entry(m, c, [&]() -> int {
        LearnedFeatures *F = c->feat;
        ICCG_CHECK(ensure_buffers(m, F->n, F->nnz, F->nl, nprobes, true));
        ICCG_CHECK(forward_fp32(m, c, true));
        ICCG_CHECK(probe_loss(m, c, probes, nprobes));
        ICCG_CHECK(backward(m, c));
        if (loss) HIP_CHECK(hipMemcpyAsync(loss, m->loss.p, sizeof(double), hipMemcpyDeviceToHost, m->work));
        if (grad) HIP_CHECK(hipMemcpyAsync(grad, m->grad.p, sizeof(float) * kL.total, hipMemcpyDeviceToHost, m->work));
        HIP_CHECK(hipStreamSynchronize(m->work));
        return ICCG_OK;
    });
}

int iccg_mpnn_train_step(iccg_mpnn *m, iccg_ctx *c, const double *probes, int nprobes, float lr,
                         double *loss) {
    if (!probes || nprobes < 1 || !(lr > 0.0f)) return set_error(ICCG_EINVAL, "need probes and lr > 0");
    return mpnn_entry(m, c, [&]() -> int {
        LearnedFeatures *F = c->feat;
        ICCG_CHECK(ensure_buffers(m, F->n, F->nnz, F->nl, nprobes, true));
        ICCG_CHECK(forward_fp32(m, c, true));
        ICCG_CHECK(probe_loss(m, c, probes, nprobes));
        ICCG_CHECK(backward(m, c));
        m->step += 1;
        // bias corrections in FP64 first: 1 - 0.999f would carry 0.999's FP32
        // representation error (1.3e-5 relative) into the first steps
        const float c1 = static_cast<float>(1.0 - std::pow(0.9, static_cast<double>(m->step)));
        const float c2 = static_cast<float>(1.0 - std::pow(0.999, static_cast<double>(m->step)));
        hipLaunchKernelGGL(k_adam, dim3(grid_of(kL.total, 256)), dim3(256), 0, m->work, kL.total, m->theta.p,
                           m->grad.p, m->m.p, m->v.p, lr, c1, c2);
        HIP_CHECK(hipGetLastError());
        if (loss) {
            HIP_CHECK(hipMemcpyAsync(loss, m->loss.p, sizeof(double), hipMemcpyDeviceToHost, m->work));
            HIP_CHECK(hipStreamSynchronize(m->work));
        }
        return ICCG_OK;
    });
}

int iccg_mpnn_predict(iccg_mpnn *m, iccg_ctx *c, int bf16_storage, double *lvals) {
    if (!lvals) return set_error(ICCG_EINVAL, "null output");
    return mpnn_entry(m, c, [&]() -> int {
        LearnedFeatures *F = c->feat;
        ICCG_CHECK(ensure_buffers(m, F->n, F->nnz, F->nl, 0, false));
        if (bf16_storage) ICCG_CHECK(forward_bf16(m, c));
        else ICCG_CHECK(forward_fp32(m, c, false));
        hipLaunchKernelGGL(k_factor_out, dim3(grid_of(F->n, 256)), dim3(256), 0, m->work, F->n, c->rowptr.p,
                           c->col.p, F->lowidx.p, c->lval0.p, F->s.p, m->delta.p, lvals);
        HIP_CHECK(hipGetLastError());
        return ICCG_OK;
    });
}

}  // extern "C"
