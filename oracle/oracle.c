/*
 * Serial FP64 CPU oracle for block-multicolored ICCG.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table or
 * helper with the GPU path.
 *
 * Everything is plain, serial and unblocked so that each step can be checked
 * against the paper by eye.  Build: gcc -O2 -ffp-contract=off -fPIC -shared.
 *
 * Paper: "Comparison of Algebraic Block Multi-Coloring and Leiden Methods for
 * Parallel Preconditioning in the ICCG Method".
 *   Section 3          ABMC blocking, block coloring, Algorithm 1 (forward
 *                      substitution), backward substitution in reverse order.
 *   Section 4, Eq. (1) modularity, Eq. (2) constant Potts model.
 *   Section 5          PCG stopping rule ||r||_2/||b||_2 <= tol, IC(0).
 *   Section 6.1        greedy block coloring, block size s = ceil(n/n_b).
 *   Section 7.1        Leiden settings; blocks sorted by descending size.
 * Leiden itself follows Traag, Waltman and van Eck (2019), the paper's
 * reference for the method (move nodes fast, refine, aggregate).
 *
 * Readings where the paper is silent are listed in the design notes; the ones
 * that change results are restated next to the code that implements them.
 *
 * Index type: int (int32).  All arrays are caller-owned unless stated.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

/* ------------------------------------------------------------------------- */
/* small utilities                                                            */
/* ------------------------------------------------------------------------- */

static void *xmalloc(size_t bytes) {
    void *p = malloc(bytes ? bytes : 1);
    if (!p) abort();
    return p;
}

static void *xcalloc(size_t count, size_t size) {
    void *p = calloc(count ? count : 1, size ? size : 1);
    if (!p) abort();
    return p;
}

static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* SplitMix64 (Steele, Lea and Flood 2014): one stream, drawn in call order. */
typedef struct { uint64_t s; } or_rng;

static uint64_t rng_next(or_rng *r) {
    uint64_t z = (r->s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Fisher-Yates: for i = len-1 down to 1, j = next() mod (i+1), swap a[i], a[j]. */
static void rng_shuffle(or_rng *r, int *a, int len) {
    for (int i = len - 1; i >= 1; --i) {
        int j = (int)(rng_next(r) % (uint64_t)(i + 1));
        int t = a[i]; a[i] = a[j]; a[j] = t;
    }
}

/* uniform double in [0,1) from the top 53 bits */
static double rng_uniform(or_rng *r) {
    return (double)(rng_next(r) >> 11) * (1.0 / 9007199254740992.0);
}

uint64_t or_splitmix64_draws(uint64_t seed, int count, uint64_t *out) {
    or_rng r = {seed};
    for (int i = 0; i < count; ++i) out[i] = rng_next(&r);
    return r.s;
}

/* ------------------------------------------------------------------------- */
/* ABMC blocking (Section 3; block size s = ceil(n/n_b), Section 6.1)         */
/* ------------------------------------------------------------------------- */
/*
 * Grow one block at a time.  A block starts from the smallest-index
 * unassigned node; nodes are taken from a FIFO candidate set that receives
 * the unassigned neighbours of each node as it joins (in ascending index).
 * When the candidate set empties before the block is full, the block is
 * re-seeded from the smallest-index unassigned node.  Candidates left over
 * when the block is full are discarded.  Every block therefore has exactly s
 * nodes except the last.
 *
 * block_of[n] receives the block id of every node; returns n_b.
 */
int or_abmc(int n, const int *rowptr, const int *col, int s, int *block_of) {
    if (n <= 0) return 0;
    if (s < 1) s = 1;
    int *queue = xmalloc(sizeof(int) * (size_t)n);
    char *inq = xcalloc((size_t)n, 1);
    for (int i = 0; i < n; ++i) block_of[i] = -1;
    int assigned = 0, seed_scan = 0, b = 0;
    while (assigned < n) {
        int head = 0, tail = 0, size = 0;
        while (size < s && assigned < n) {
            int v;
            if (head == tail) {
                while (block_of[seed_scan] >= 0) ++seed_scan;
                v = seed_scan;
            } else {
                v = queue[head++];
            }
            block_of[v] = b;
            ++size;
            ++assigned;
            for (int k = rowptr[v]; k < rowptr[v + 1]; ++k) {
                int u = col[k];
                if (u == v) continue;
                if (block_of[u] < 0 && !inq[u]) {
                    inq[u] = 1;
                    queue[tail++] = u;
                }
            }
        }
        for (int q = 0; q < tail; ++q) inq[queue[q]] = 0;
        ++b;
    }
    free(queue);
    free(inq);
    return b;
}

/* ------------------------------------------------------------------------- */
/* Greedy block coloring (Section 3, Section 6.1)                             */
/* ------------------------------------------------------------------------- */
/*
 * Blocks b != b' are adjacent when a stored entry a_ij has i in b, j in b'.
 * Blocks are visited in ascending id and take the smallest color not used by
 * an already-colored adjacent block.  Returns n_c.
 */
int or_color_blocks(int n, const int *rowptr, const int *col, int nb,
                    const int *block_of, int *color_of_block) {
    if (nb <= 0) return 0;
    /* members of each block, ascending node index */
    int *bptr = xcalloc((size_t)nb + 1, sizeof(int));
    for (int i = 0; i < n; ++i) bptr[block_of[i] + 1]++;
    for (int b = 0; b < nb; ++b) bptr[b + 1] += bptr[b];
    int *fill = xmalloc(sizeof(int) * (size_t)nb);
    memcpy(fill, bptr, sizeof(int) * (size_t)nb);
    int *mem = xmalloc(sizeof(int) * (size_t)n);
    for (int i = 0; i < n; ++i) mem[fill[block_of[i]]++] = i;

    int *mark = xmalloc(sizeof(int) * ((size_t)nb + 1));
    for (int c = 0; c <= nb; ++c) mark[c] = -1;
    for (int b = 0; b < nb; ++b) color_of_block[b] = -1;
    int nc = 0;
    for (int b = 0; b < nb; ++b) {
        for (int m = bptr[b]; m < bptr[b + 1]; ++m) {
            int i = mem[m];
            for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                int bb = block_of[col[k]];
                if (bb != b && color_of_block[bb] >= 0) mark[color_of_block[bb]] = b;
            }
        }
        int c = 0;
        while (mark[c] == b) ++c;
        color_of_block[b] = c;
        if (c + 1 > nc) nc = c + 1;
    }
    free(bptr); free(fill); free(mem); free(mark);
    return nc;
}

/* ------------------------------------------------------------------------- */
/* Color-major ordering (Algorithm 1 processes colors in sequence; Section    */
/* 7.1 keeps each block in a contiguous index range)                          */
/* ------------------------------------------------------------------------- */
/*
 * New numbering: colors ascending, then the blocks of that color in ascending
 * block id, then the rows of a block in ascending original index.
 * perm[new] = old; block_ptr[k] = first new row of the k-th block in this
 * order (size n_b+1); color_ptr[c] = first block (in this order) of color c
 * (size n_c+1).
 */
void or_order(int n, int nb, const int *block_of, const int *color_of_block, int nc,
              int *perm, int *block_ptr, int *color_ptr) {
    int *bsize = xcalloc((size_t)nb, sizeof(int));
    for (int i = 0; i < n; ++i) bsize[block_of[i]]++;
    int *seq = xmalloc(sizeof(int) * (size_t)(nb ? nb : 1));   /* block ids in new order */
    int k = 0;
    for (int c = 0; c < nc; ++c) {
        color_ptr[c] = k;
        for (int b = 0; b < nb; ++b)
            if (color_of_block[b] == c) seq[k++] = b;
    }
    color_ptr[nc] = k;
    int *start = xmalloc(sizeof(int) * (size_t)(nb ? nb : 1));  /* by block id */
    int pos = 0;
    for (int q = 0; q < nb; ++q) {
        block_ptr[q] = pos;
        start[seq[q]] = pos;
        pos += bsize[seq[q]];
    }
    block_ptr[nb] = pos;
    for (int i = 0; i < n; ++i) perm[start[block_of[i]]++] = i;   /* ascending i */
    free(bsize); free(seq); free(start);
}

/* ------------------------------------------------------------------------- */
/* Symmetric permutation A' = P A P^T, columns sorted                         */
/* ------------------------------------------------------------------------- */
void or_permute(int n, const int *rowptr, const int *col, const double *val,
                const int *perm, int *prow, int *pcol, double *pval) {
    int *iperm = xmalloc(sizeof(int) * (size_t)n);
    for (int i = 0; i < n; ++i) iperm[perm[i]] = i;
    prow[0] = 0;
    for (int i = 0; i < n; ++i) {
        int o = perm[i];
        int base = prow[i];
        int len = rowptr[o + 1] - rowptr[o];
        for (int t = 0; t < len; ++t) {
            /* insertion sort by new column index */
            int c = iperm[col[rowptr[o] + t]];
            double v = val[rowptr[o] + t];
            int p = base + t;
            while (p > base && pcol[p - 1] > c) {
                pcol[p] = pcol[p - 1];
                pval[p] = pval[p - 1];
                --p;
            }
            pcol[p] = c;
            pval[p] = v;
        }
        prow[i + 1] = base + len;
    }
    free(iperm);
}

/* ------------------------------------------------------------------------- */
/* IC(0) factorization, A' ~= L L^T with pattern(L) = lower(A') (Section 3)   */
/* ------------------------------------------------------------------------- */
/*
 * Row by row, i = 0..n-1:
 *   for each k < i in pattern(i), ascending:
 *       L_ik = (a_ik - sum_{j<k, j in pattern(i) and pattern(k)} L_ij L_kj) / L_kk
 *   L_ii = sqrt(a_ii - sum_{k<i} L_ik^2)
 * Each sum is taken as a running subtraction from a_ik (a_ii) in ascending j
 * (k), the same way Algorithm 1 accumulates s.
 *
 * lval[nnz] receives L at the positions of A's lower triangle including the
 * diagonal; upper positions are set to 0.  Returns -1 on success or the row
 * at which the pivot a_ii - sum L_ik^2 was not > 0 (or not finite).
 */
int or_ic0(int n, const int *rowptr, const int *col, const double *val, double *lval) {
    int nnz = rowptr[n];
    for (int k = 0; k < nnz; ++k) lval[k] = 0.0;
    int *dpos = xmalloc(sizeof(int) * (size_t)(n ? n : 1));
    for (int i = 0; i < n; ++i) {
        dpos[i] = -1;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
            if (col[k] == i) dpos[i] = k;
        if (dpos[i] < 0) { free(dpos); return i; }
    }
    for (int i = 0; i < n; ++i) {
        for (int p = rowptr[i]; p < dpos[i]; ++p) {
            int k = col[p];
            double s = val[p];
            /* merge row i (entries j<k) with row k (entries j<k) */
            int a = rowptr[i], b = rowptr[k];
            while (a < p && b < dpos[k]) {
                if (col[a] < col[b]) ++a;
                else if (col[a] > col[b]) ++b;
                else { s -= lval[a] * lval[b]; ++a; ++b; }
            }
            lval[p] = s / lval[dpos[k]];
        }
        double d = val[dpos[i]];
        for (int p = rowptr[i]; p < dpos[i]; ++p) d -= lval[p] * lval[p];
        if (!(d > 0.0) || !isfinite(d)) { free(dpos); return i; }
        lval[dpos[i]] = sqrt(d);
    }
    free(dpos);
    return -1;
}

/* ------------------------------------------------------------------------- */
/* Triangular solves in serial row order                                      */
/* ------------------------------------------------------------------------- */
/*
 * Forward substitution L y = r (Algorithm 1 run serially over the new
 * numbering): s = r_i; s -= L_ij y_j for j < i ascending; y_i = s / L_ii.
 * Color-major numbering with no edge between same-colored blocks makes this
 * identical (in exact arithmetic) to the block-parallel schedule.
 */
void or_forward(int n, const int *rowptr, const int *col, const double *lval,
                const double *r, double *y) {
    for (int i = 0; i < n; ++i) {
        double s = r[i];
        double d = 0.0;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            int j = col[k];
            if (j < i) s -= lval[k] * y[j];
            else if (j == i) d = lval[k];
        }
        y[i] = s / d;
    }
}

static int find_in_row(const int *rowptr, const int *col, int row, int c) {
    int lo = rowptr[row], hi = rowptr[row + 1] - 1;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        if (col[mid] == c) return mid;
        if (col[mid] < c) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/*
 * Backward substitution L^T z = y (Section 3: same scheme, colors and the
 * rows of each block in reverse order; serially this is i = n-1 down to 0):
 * s = y_i; s -= L_ji z_j for j > i ascending; z_i = s / L_ii.
 * L_ji is found at position (j, i) of the symmetric pattern.
 */
void or_backward(int n, const int *rowptr, const int *col, const double *lval,
                 const double *y, double *z) {
    for (int i = n - 1; i >= 0; --i) {
        double s = y[i];
        double d = 0.0;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            int j = col[k];
            if (j > i) {
                int q = find_in_row(rowptr, col, j, i);
                s -= lval[q] * z[j];
            } else if (j == i) {
                d = lval[k];
            }
        }
        z[i] = s / d;
    }
}

/* z = (L L^T)^{-1} r */
void or_ic_apply(int n, const int *rowptr, const int *col, const double *lval,
                 const double *r, double *z) {
    double *y = xmalloc(sizeof(double) * (size_t)(n ? n : 1));
    or_forward(n, rowptr, col, lval, r, y);
    or_backward(n, rowptr, col, lval, y, z);
    free(y);
}

void or_spmv(int n, const int *rowptr, const int *col, const double *val,
             const double *x, double *y) {
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) s += val[k] * x[col[k]];
        y[i] = s;
    }
}

double or_dot(int n, const double *a, const double *b) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* ------------------------------------------------------------------------- */
/* Preconditioned CG (Section 5: stop when ||r||_2 / ||b||_2 <= tol)          */
/* ------------------------------------------------------------------------- */
/*
 *   x = x0; r = b - A x; z = M^{-1} r; p = z; rho = (r, z)
 *   if ||r||/||b|| <= tol: done after 0 iterations
 *   for k = 1..maxit:
 *       q = A p; alpha = rho / (p, q); x += alpha p; r -= alpha q
 *       if ||r||/||b|| <= tol: done after k iterations
 *       z = M^{-1} r; rho' = (r, z); beta = rho'/rho; rho = rho'; p = z + beta p
 * M = L L^T when lval is given, identity when lval is NULL.
 *
 * x: in x0, out the last iterate.  Outputs: *iters, *relres (recursive),
 * *relres_true (||b - A x|| / ||b||), hist[k] = recursive relres after
 * iteration k (hist[0] the initial one; size maxit+1), alphas/betas (size
 * maxit, may be NULL), phase[4] = seconds in forward substitution, backward
 * substitution, SpMV and everything else (may be NULL).
 * Returns 0 converged, 1 maxit reached, 2 (p,q) <= 0 or non-finite.
 */
int or_pcg(int n, const int *rowptr, const int *col, const double *val,
           const double *lval, const double *b, double *x, double tol, int maxit,
           int *iters, double *relres, double *relres_true, double *hist,
           double *alphas, double *betas, double *phase) {
    size_t bytes = sizeof(double) * (size_t)(n ? n : 1);
    double *r = xmalloc(bytes), *z = xmalloc(bytes), *p = xmalloc(bytes);
    double *q = xmalloc(bytes), *y = xmalloc(bytes);
    double tf = 0, tb = 0, ts = 0, t_all0 = now_s(), t0;
    int status = 1, k = 0;

    t0 = now_s();
    or_spmv(n, rowptr, col, val, x, q);
    ts += now_s() - t0;
    for (int i = 0; i < n; ++i) r[i] = b[i] - q[i];
    double bnorm = sqrt(or_dot(n, b, b));
    if (bnorm == 0.0) bnorm = 1.0;
    double res = sqrt(or_dot(n, r, r)) / bnorm;
    if (hist) hist[0] = res;
    if (res <= tol) { status = 0; goto done; }
    if (lval) {
        t0 = now_s(); or_forward(n, rowptr, col, lval, r, y); tf += now_s() - t0;
        t0 = now_s(); or_backward(n, rowptr, col, lval, y, z); tb += now_s() - t0;
    } else {
        memcpy(z, r, bytes);
    }
    memcpy(p, z, bytes);
    double rho = or_dot(n, r, z);
    for (k = 1; k <= maxit; ++k) {
        t0 = now_s();
        or_spmv(n, rowptr, col, val, p, q);
        ts += now_s() - t0;
        double pq = or_dot(n, p, q);
        if (!(pq > 0.0) || !isfinite(pq)) { status = 2; --k; break; }
        double alpha = rho / pq;
        if (alphas) alphas[k - 1] = alpha;
        for (int i = 0; i < n; ++i) x[i] += alpha * p[i];
        for (int i = 0; i < n; ++i) r[i] -= alpha * q[i];
        res = sqrt(or_dot(n, r, r)) / bnorm;
        if (hist) hist[k] = res;
        if (res <= tol) { status = 0; break; }
        if (k == maxit) break;
        if (lval) {
            t0 = now_s(); or_forward(n, rowptr, col, lval, r, y); tf += now_s() - t0;
            t0 = now_s(); or_backward(n, rowptr, col, lval, y, z); tb += now_s() - t0;
        } else {
            memcpy(z, r, bytes);
        }
        double rho2 = or_dot(n, r, z);
        double beta = rho2 / rho;
        if (betas) betas[k - 1] = beta;
        rho = rho2;
        for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
    if (k > maxit) k = maxit;
done:
    *iters = k;
    *relres = res;
    or_spmv(n, rowptr, col, val, x, q);
    for (int i = 0; i < n; ++i) r[i] = b[i] - q[i];
    *relres_true = sqrt(or_dot(n, r, r)) / bnorm;
    if (phase) {
        phase[0] = tf; phase[1] = tb; phase[2] = ts;
        phase[3] = (now_s() - t_all0) - tf - tb - ts;
    }
    free(r); free(z); free(p); free(q); free(y);
    return status;
}

/* ------------------------------------------------------------------------- */
/* Leiden community detection (Section 4; Traag, Waltman, van Eck 2019)       */
/* ------------------------------------------------------------------------- */
/*
 * Quality functions.  Both Eq. (1) and Eq. (2) change, when an isolated node
 * v (node weight a) joins community C (node weight b), by 2/(2m) times
 *     dH = w(v, C) - pen(a, b),
 * with pen(a, b) = gamma * a * b for CPM (node weight = number of original
 * nodes) and pen(a, b) = gamma * a * b / (2m) for modularity (node weight =
 * summed original degree).  dH is evaluated exactly as
 *     (double)w - ((gamma * (double)a) * (double)b) [/ (double)twom]
 * with integer w, a, b; the argmax is that of the quality change.
 * The graph is the unweighted pattern graph of A (edge {i,j} for every stored
 * a_ij with i != j); aggregated edge weights are integer sums.
 */
typedef struct {
    int n;
    int64_t *ptr;     /* n+1 */
    int *adj;         /* neighbours, ascending, no self loops */
    int64_t *w;       /* edge weights */
    int64_t *nw;      /* node weights */
} lg_graph;

static void lg_free(lg_graph *g) {
    free(g->ptr); free(g->adj); free(g->w); free(g->nw);
    memset(g, 0, sizeof(*g));
}

typedef struct {
    int quality;      /* 0 = modularity, 1 = CPM */
    double gamma;
    double twom;
} lg_q;

static double lg_pen(const lg_q *q, int64_t a, int64_t b) {
    double t = (q->gamma * (double)a) * (double)b;
    if (q->quality == 0) t = t / q->twom;
    return t;
}

/* binary min-heap of community ids, lazy deletion (entries may be stale) */
typedef struct { int *a; int len, cap; } lg_heap;

static void heap_push(lg_heap *h, int v) {
    if (h->len == h->cap) {
        h->cap = h->cap ? 2 * h->cap : 64;
        h->a = realloc(h->a, sizeof(int) * (size_t)h->cap);
        if (!h->a) abort();
    }
    int i = h->len++;
    h->a[i] = v;
    while (i > 0) {
        int p = (i - 1) / 2;
        if (h->a[p] <= h->a[i]) break;
        int t = h->a[p]; h->a[p] = h->a[i]; h->a[i] = t;
        i = p;
    }
}

static void heap_pop(lg_heap *h) {
    h->a[0] = h->a[--h->len];
    int i = 0;
    for (;;) {
        int l = 2 * i + 1, r = l + 1, m = i;
        if (l < h->len && h->a[l] < h->a[m]) m = l;
        if (r < h->len && h->a[r] < h->a[m]) m = r;
        if (m == i) break;
        int t = h->a[m]; h->a[m] = h->a[i]; h->a[i] = t;
        i = m;
    }
}

static int cmp_int(const void *a, const void *b) {
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/*
 * Move nodes fast.  Queue = random permutation of the nodes.  Pop v, take it
 * out of its community D, and evaluate dH for D (the incumbent), for every
 * community adjacent to v in ascending id (a candidate wins only when strictly
 * better), and finally for an empty community (dH = 0; the smallest empty id
 * is used).  Insert v into the winner; if it moved, append to the queue every
 * neighbour (ascending) that is outside the new community and not queued.
 */
static void lg_move_nodes(const lg_graph *g, int *comm, const lg_q *q, or_rng *rng) {
    int n = g->n;
    int64_t *csize = xcalloc((size_t)n, sizeof(int64_t));
    int *ccount = xcalloc((size_t)n, sizeof(int));
    for (int v = 0; v < n; ++v) { csize[comm[v]] += g->nw[v]; ccount[comm[v]]++; }
    lg_heap empty = {0};
    for (int c = 0; c < n; ++c) if (ccount[c] == 0) heap_push(&empty, c);

    int *queue = xmalloc(sizeof(int) * (size_t)n);
    char *inq = xmalloc((size_t)n);
    for (int v = 0; v < n; ++v) { queue[v] = v; inq[v] = 1; }
    rng_shuffle(rng, queue, n);
    int head = 0, count = n;    /* circular buffer of capacity n */

    int64_t *wsum = xcalloc((size_t)n, sizeof(int64_t));
    int *stamp = xmalloc(sizeof(int) * (size_t)n);
    for (int c = 0; c < n; ++c) stamp[c] = -1;
    int *touched = xmalloc(sizeof(int) * (size_t)n);

    while (count > 0) {
        int v = queue[head];
        head = (head + 1) % n;
        --count;
        inq[v] = 0;
        int D = comm[v];
        int nt = 0;
        for (int64_t e = g->ptr[v]; e < g->ptr[v + 1]; ++e) {
            int c = comm[g->adj[e]];
            if (stamp[c] != v) { stamp[c] = v; wsum[c] = 0; touched[nt++] = c; }
            wsum[c] += g->w[e];
        }
        csize[D] -= g->nw[v];
        ccount[D]--;
        if (ccount[D] == 0) heap_push(&empty, D);
        int64_t wD = (stamp[D] == v) ? wsum[D] : 0;
        int best = D;
        double bestH = (double)wD - lg_pen(q, g->nw[v], csize[D]);
        qsort(touched, (size_t)nt, sizeof(int), cmp_int);
        for (int t = 0; t < nt; ++t) {
            int c = touched[t];
            if (c == D) continue;
            double h = (double)wsum[c] - lg_pen(q, g->nw[v], csize[c]);
            if (h > bestH) { best = c; bestH = h; }
        }
        if (0.0 > bestH) {
            while (ccount[empty.a[0]] != 0) heap_pop(&empty);
            best = empty.a[0];
            bestH = 0.0;
        }
        csize[best] += g->nw[v];
        ccount[best]++;
        comm[v] = best;
        if (best != D) {
            for (int64_t e = g->ptr[v]; e < g->ptr[v + 1]; ++e) {
                int u = g->adj[e];
                if (comm[u] != best && !inq[u]) {
                    inq[u] = 1;
                    queue[(head + count) % n] = u;
                    ++count;
                }
            }
        }
    }
    free(csize); free(ccount); free(empty.a); free(queue); free(inq);
    free(wsum); free(stamp); free(touched);
}

/*
 * Refinement.  Start from singletons.  For every community S of the moved
 * partition, in ascending id: the well-connected nodes of S are those with
 * E(v, S - v) >= pen(|v|, |S| - |v|); visit them in a random order (Fisher-
 * Yates of their ascending list).  A visited node that is still a singleton
 * considers its own singleton (dH = 0) and every refined community C inside S
 * adjacent to it that is itself well connected, E(C, S - C) >= pen(|C|,
 * |S| - |C|).  Of the candidates with dH >= 0 it picks C with probability
 * proportional to exp((dH_C - dH_max) / beta): one uniform draw u, the first
 * candidate (ascending id) whose running sum reaches u * total.
 *
 * rcomm[v] receives the refined community id (a node id of S).
 */
static void lg_refine(const lg_graph *g, const int *comm, int *rcomm, const lg_q *q,
                      double beta, or_rng *rng) {
    int n = g->n;
    int64_t *rsize = xmalloc(sizeof(int64_t) * (size_t)n);
    int *rcount = xmalloc(sizeof(int) * (size_t)n);
    int64_t *rext = xmalloc(sizeof(int64_t) * (size_t)n);
    int64_t *ext = xmalloc(sizeof(int64_t) * (size_t)n);
    for (int v = 0; v < n; ++v) { rcomm[v] = v; rsize[v] = g->nw[v]; rcount[v] = 1; }

    /* members of every community, ascending */
    int *cptr = xcalloc((size_t)n + 1, sizeof(int));
    for (int v = 0; v < n; ++v) cptr[comm[v] + 1]++;
    for (int c = 0; c < n; ++c) cptr[c + 1] += cptr[c];
    int *fill = xmalloc(sizeof(int) * (size_t)n);
    memcpy(fill, cptr, sizeof(int) * (size_t)n);
    int *mem = xmalloc(sizeof(int) * (size_t)n);
    for (int v = 0; v < n; ++v) mem[fill[comm[v]]++] = v;
    int64_t *stot = xcalloc((size_t)n, sizeof(int64_t));
    for (int v = 0; v < n; ++v) stot[comm[v]] += g->nw[v];

    int64_t *wsum = xcalloc((size_t)n, sizeof(int64_t));
    int *stamp = xmalloc(sizeof(int) * (size_t)n);
    for (int c = 0; c < n; ++c) stamp[c] = -1;
    int *touched = xmalloc(sizeof(int) * (size_t)n);
    int *R = xmalloc(sizeof(int) * (size_t)n);
    double *hval = xmalloc(sizeof(double) * (size_t)n);
    int *cand = xmalloc(sizeof(int) * (size_t)n);

    for (int S = 0; S < n; ++S) {
        if (cptr[S] == cptr[S + 1]) continue;
        int64_t NS = stot[S];
        int nr = 0;
        for (int m = cptr[S]; m < cptr[S + 1]; ++m) {
            int v = mem[m];
            int64_t e_in = 0;
            for (int64_t e = g->ptr[v]; e < g->ptr[v + 1]; ++e)
                if (comm[g->adj[e]] == S) e_in += g->w[e];
            ext[v] = e_in;
            rext[v] = e_in;
            if ((double)e_in >= lg_pen(q, g->nw[v], NS - g->nw[v])) R[nr++] = v;
        }
        rng_shuffle(rng, R, nr);
        for (int t = 0; t < nr; ++t) {
            int v = R[t];
            if (rcount[rcomm[v]] != 1) continue;     /* no longer a singleton */
            int nt = 0;
            for (int64_t e = g->ptr[v]; e < g->ptr[v + 1]; ++e) {
                int u = g->adj[e];
                if (comm[u] != S) continue;
                int c = rcomm[u];
                if (stamp[c] != v) { stamp[c] = v; wsum[c] = 0; touched[nt++] = c; }
                wsum[c] += g->w[e];
            }
            /* take v out of its singleton (own id v, dH = 0) */
            int nc = 0;
            cand[nc] = v; hval[nc] = 0.0; ++nc;
            for (int k = 0; k < nt; ++k) {
                int c = touched[k];
                if (c == v) continue;
                if (!((double)rext[c] >= lg_pen(q, rsize[c], NS - rsize[c]))) continue;
                double h = (double)wsum[c] - lg_pen(q, g->nw[v], rsize[c]);
                if (h >= 0.0) { cand[nc] = c; hval[nc] = h; ++nc; }
            }
            /* ascending id: sort (cand, hval) pairs by cand */
            for (int a = 1; a < nc; ++a) {
                int ci = cand[a]; double hi = hval[a]; int p = a;
                while (p > 0 && cand[p - 1] > ci) { cand[p] = cand[p - 1]; hval[p] = hval[p - 1]; --p; }
                cand[p] = ci; hval[p] = hi;
            }
            double hmax = hval[0];
            for (int a = 1; a < nc; ++a) if (hval[a] > hmax) hmax = hval[a];
            double total = 0.0;
            for (int a = 0; a < nc; ++a) total += exp((hval[a] - hmax) / beta);
            double u = rng_uniform(rng) * total;
            double cum = 0.0;
            int pick = cand[nc - 1];
            for (int a = 0; a < nc; ++a) {
                cum += exp((hval[a] - hmax) / beta);
                if (cum >= u) { pick = cand[a]; break; }
            }
            if (pick != v) {
                int64_t wvc = (stamp[pick] == v) ? wsum[pick] : 0;
                rcount[v] = 0;
                rsize[v] = 0;
                rcomm[v] = pick;
                rcount[pick]++;
                rsize[pick] += g->nw[v];
                rext[pick] = rext[pick] + ext[v] - 2 * wvc;
            }
        }
    }
    free(rsize); free(rcount); free(rext); free(ext); free(cptr); free(fill); free(mem);
    free(stot); free(wsum); free(stamp); free(touched); free(R); free(hval); free(cand);
}

/* Renumber a partition of n nodes (ids in [0, idrange)) to 0..k-1 in
 * ascending order of each community's smallest member.  Returns k. */
static int lg_canonical(int n, int *comm, int idrange) {
    int *map = xmalloc(sizeof(int) * (size_t)(idrange ? idrange : 1));
    for (int c = 0; c < idrange; ++c) map[c] = -1;
    int k = 0;
    for (int v = 0; v < n; ++v) {
        if (map[comm[v]] < 0) map[comm[v]] = k++;
        comm[v] = map[comm[v]];
    }
    free(map);
    return k;
}

typedef struct { int a, b; int64_t w; } lg_edge;

static int cmp_edge(const void *x, const void *y) {
    const lg_edge *e = x, *f = y;
    if (e->a != f->a) return (e->a > f->a) - (e->a < f->a);
    return (e->b > f->b) - (e->b < f->b);
}

/*
 * Aggregate: one node per refined community, numbered in ascending order of
 * its smallest member (map[v] = aggregate node of v).  Node weights and edge
 * weights are summed; edges inside a refined community disappear (they only
 * ever add to a self loop, which no gain or connectivity test uses).
 */
static void lg_aggregate(const lg_graph *g, const int *map, int k, lg_graph *out) {
    int64_t ne = g->ptr[g->n];
    lg_edge *es = xmalloc(sizeof(lg_edge) * (size_t)(ne ? ne : 1));
    int64_t m = 0;
    for (int v = 0; v < g->n; ++v)
        for (int64_t e = g->ptr[v]; e < g->ptr[v + 1]; ++e) {
            int a = map[v], b = map[g->adj[e]];
            if (a == b) continue;
            es[m].a = a; es[m].b = b; es[m].w = g->w[e]; ++m;
        }
    qsort(es, (size_t)m, sizeof(lg_edge), cmp_edge);
    out->n = k;
    out->ptr = xcalloc((size_t)k + 1, sizeof(int64_t));
    out->adj = xmalloc(sizeof(int) * (size_t)(m ? m : 1));
    out->w = xmalloc(sizeof(int64_t) * (size_t)(m ? m : 1));
    out->nw = xcalloc((size_t)k, sizeof(int64_t));
    for (int v = 0; v < g->n; ++v) out->nw[map[v]] += g->nw[v];
    /* merge equal (a, b) pairs; the edges are sorted, so rows come out in order */
    int64_t cnt = 0;
    for (int64_t t = 0; t < m; ++t) {
        if (t > 0 && es[t].a == es[t - 1].a && es[t].b == es[t - 1].b) {
            out->w[cnt - 1] += es[t].w;
        } else {
            out->adj[cnt] = es[t].b;
            out->w[cnt] = es[t].w;
            out->ptr[es[t].a + 1]++;
            ++cnt;
        }
    }
    for (int a = 0; a < k; ++a) out->ptr[a + 1] += out->ptr[a];
    free(es);
}

/*
 * Full Leiden run.  membership[n] receives the communities numbered in
 * ascending order of their smallest node.  Returns the number of
 * communities.
 *
 *   P = singletons
 *   repeat n_iter times:
 *       G_l = G; P_l = P
 *       loop:
 *           move nodes fast on (G_l, P_l)
 *           stop if every community of P_l is a single node of G_l
 *           R = refine(G_l, P_l)
 *           stop if R is all singletons (aggregation would not shrink G_l)
 *           G_l = aggregate(G_l, R); P_l = P_l induced on the aggregate nodes
 *       P = P_l carried back to the original nodes
 */
int or_leiden(int n, const int *rowptr, const int *col, int quality, double gamma,
              double beta, int n_iter, uint64_t seed, int *membership) {
    if (n <= 0) return 0;
    or_rng rng = {seed};
    /* level-0 graph: unweighted pattern graph */
    lg_graph g0;
    g0.n = n;
    g0.ptr = xcalloc((size_t)n + 1, sizeof(int64_t));
    for (int i = 0; i < n; ++i) {
        int64_t d = 0;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) if (col[k] != i) ++d;
        g0.ptr[i + 1] = g0.ptr[i] + d;
    }
    int64_t ne = g0.ptr[n];
    g0.adj = xmalloc(sizeof(int) * (size_t)(ne ? ne : 1));
    g0.w = xmalloc(sizeof(int64_t) * (size_t)(ne ? ne : 1));
    g0.nw = xmalloc(sizeof(int64_t) * (size_t)n);
    for (int i = 0; i < n; ++i) {
        int64_t p = g0.ptr[i];
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
            if (col[k] != i) { g0.adj[p] = col[k]; g0.w[p] = 1; ++p; }
        g0.nw[i] = (quality == 0) ? (g0.ptr[i + 1] - g0.ptr[i]) : 1;
    }
    lg_q q = {quality, gamma, (double)ne};

    for (int i = 0; i < n; ++i) membership[i] = i;
    int *node_of = xmalloc(sizeof(int) * (size_t)n);   /* original -> current level node */
    for (int it = 0; it < n_iter; ++it) {
        lg_graph cur = g0;       /* borrowed at level 0 */
        int owned = 0;
        int *comm = xmalloc(sizeof(int) * (size_t)n);
        memcpy(comm, membership, sizeof(int) * (size_t)n);
        for (int i = 0; i < n; ++i) node_of[i] = i;
        for (;;) {
            lg_move_nodes(&cur, comm, &q, &rng);
            int ncomm = 0;
            {
                char *seen = xcalloc((size_t)cur.n, 1);
                for (int v = 0; v < cur.n; ++v) if (!seen[comm[v]]) { seen[comm[v]] = 1; ++ncomm; }
                free(seen);
            }
            if (ncomm == cur.n) break;
            int *rcomm = xmalloc(sizeof(int) * (size_t)cur.n);
            lg_refine(&cur, comm, rcomm, &q, beta, &rng);
            int k = lg_canonical(cur.n, rcomm, cur.n);      /* rcomm[v] = aggregate node of v */
            if (k == cur.n) { free(rcomm); break; }
            lg_graph nxt;
            lg_aggregate(&cur, rcomm, k, &nxt);
            int *ncomm_arr = xmalloc(sizeof(int) * (size_t)k);
            for (int v = 0; v < cur.n; ++v) ncomm_arr[rcomm[v]] = comm[v];
            lg_canonical(k, ncomm_arr, cur.n);
            for (int i = 0; i < n; ++i) node_of[i] = rcomm[node_of[i]];
            free(rcomm);
            free(comm);
            comm = ncomm_arr;
            if (owned) lg_free(&cur);
            cur = nxt;
            owned = 1;
        }
        for (int i = 0; i < n; ++i) membership[i] = comm[node_of[i]];
        lg_canonical(n, membership, cur.n);
        free(comm);
        if (owned) lg_free(&cur);
    }
    free(node_of);
    int k = 0;
    for (int i = 0; i < n; ++i) if (membership[i] + 1 > k) k = membership[i] + 1;
    lg_free(&g0);
    return k;
}

/*
 * Block numbering for Leiden blocks (Section 7.1): descending size; ties go
 * to the block with the smaller minimum original node index.  Renumbers
 * block_of in place.
 */
typedef struct { int id, size, minv; } sb_key;

static int cmp_sb(const void *x, const void *y) {
    const sb_key *a = x, *b = y;
    if (a->size != b->size) return (a->size < b->size) - (a->size > b->size);
    return (a->minv > b->minv) - (a->minv < b->minv);
}

void or_sort_blocks(int n, int nb, int *block_of) {
    sb_key *keys = xmalloc(sizeof(sb_key) * (size_t)(nb ? nb : 1));
    for (int b = 0; b < nb; ++b) { keys[b].id = b; keys[b].size = 0; keys[b].minv = n; }
    for (int i = 0; i < n; ++i) {
        sb_key *k = &keys[block_of[i]];
        k->size++;
        if (i < k->minv) k->minv = i;
    }
    qsort(keys, (size_t)nb, sizeof(sb_key), cmp_sb);
    int *newid = xmalloc(sizeof(int) * (size_t)(nb ? nb : 1));
    for (int r = 0; r < nb; ++r) newid[keys[r].id] = r;
    for (int i = 0; i < n; ++i) block_of[i] = newid[block_of[i]];
    free(keys); free(newid);
}
