/*
 * CPU oracle for synchronous parallel Louvain -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded C implementation of what the method
 * computes, written from R. Forster, "Parallel Louvain Community Detection
 * Optimized for GPUs" (arXiv 1805.10904).  Only the test-suite, the smoke
 * check and the benchmark's CPU-baseline leg load it; the GPU library never
 * links, calls or includes anything from here, and this file includes
 * nothing from the GPU library.
 *
 * Conventions (the paper's Section 2 problem statement, read as an
 * adjacency matrix A):
 *   - The graph is a symmetric CSR: entry (i, j, w) is A_ij = w, and an
 *     undirected edge {i, j}, i != j, is stored in rows i and j.  A loop is
 *     stored once, as A_ii.  Weights are integers >= 1.
 *   - delta_i = sum_j A_ij (the weighted degree; a loop counts once), and
 *     TW = 2W = sum_i delta_i.
 *   - e_{i->C} = sum_{j in C} A_ij (eq. 1), deg_C = sum_{i in C} delta_i
 *     (eq. 2), and modularity (eq. 3) is kept as the exact integer
 *     Q_int = TW^2 * Q = TW * sum_i e_{i->C(i)} - sum_C deg_C^2.
 *   - The gain of moving i into C (eq. 4) is compared as the integer score
 *     s(C) = TW * e_{i->C} - delta_i * deg_C, with i's own community
 *     scored without i: s_own = TW * e_{i->C(i)\{i}} - delta_i *
 *     (deg_{C(i)} - delta_i).  Then dQ_{i->C} = 2 (s(C) - s_own) / TW^2.
 *     Loops are left out of e_{i->C} in this score (the paper zeroes the
 *     weight of loop edges before evaluating moves).
 *   - Moves (eq. 5 with the two heuristics of Section 3.1): the candidate
 *     with the largest s(C), ties to the smallest label (generalized minimum
 *     label heuristic); move only if that score beats s_own strictly; a
 *     singleton vertex does not move into another singleton community with
 *     a larger label (singlet minimum label heuristic) and then stays.
 *   - Sweeps are synchronous (Alg. 1): every vertex decides from the
 *     previous sweep's labels, degrees and sizes.  A sweep is kept iff
 *     theta_den * (Q_new - Q_prev) > theta_num * |Q_prev| (exact); otherwise
 *     it is discarded and the phase ends.
 *   - Final merge (optional; Section 5.1, end of "Generating one level":
 *     after the last iteration, vertices with a single neighbouring
 *     community are pushed into it).  Read here as one more synchronous
 *     decision, made from the phase's final labels, for vertices alone in
 *     their community whose neighbours (loops aside) all carry one label C:
 *     such a vertex joins C iff s(C) beats s_own strictly and the singlet
 *     rule allows it, as in a sweep.  It is applied without the acceptance
 *     test, only after a phase that kept a sweep, and Q is recomputed.
 *   - Phases (Alg. 2): after a phase that kept at least one sweep, the
 *     labels are renumbered densely in ascending label order and the graph
 *     is contracted: A'_ab = sum of A_ij over i in a, j in b (a loop of a
 *     super-vertex is the sum over both directions of its internal edges
 *     plus its members' loops).  The driver stops after a phase that kept
 *     no sweep.
 *
 * All decisions use exact integer arithmetic (int64 sums, 128-bit
 * products); the only floating-point value is the reported Q.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#define THREAD_ID() omp_get_thread_num()
#else
#define THREAD_ID() 0
#endif

typedef __int128 i128;
typedef unsigned __int128 u128;

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_ELIMIT = -6 };

/* Threads of the OpenMP variant: the sweep's vertex loop and the inner
 * weight of eq. 3 run over this many threads (1 = the plain single-threaded
 * oracle).  Every vertex decides from the same snapshot and the sums are of
 * integers, so results do not depend on the count. */
static int g_threads = 1;

void orc_set_threads(int threads)
{
    g_threads = threads < 1 ? 1 : threads;
}

int orc_get_threads(void)
{
    return g_threads;
}

/* Weighted degrees delta_i and TW = sum_i delta_i (Section 2). */
int orc_degrees(int64_t n, const int64_t *row_ptr, const int64_t *w,
                int64_t *delta, int64_t *tw)
{
    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t s = 0;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
            s += w[e];
        delta[i] = s;
        total += s;
    }
    *tw = total;
    return ORC_OK;
}

static void put_i128(i128 v, int64_t out[2])
{
    u128 u = (u128)v;
    out[0] = (int64_t)(uint64_t)u;          /* low 64 bits  */
    out[1] = (int64_t)(uint64_t)(u >> 64);  /* high 64 bits */
}

static i128 get_i128(const int64_t in[2])
{
    u128 u = ((u128)(uint64_t)in[1] << 64) | (u128)(uint64_t)in[0];
    return (i128)u;
}

/* Q_int = TW * sum_i e_{i->C(i)} - sum_C deg_C^2 (eq. 3 times TW^2); labels
 * must lie in [0, n).  Loops count in e_{i->C(i)}. */
static i128 modularity_int(int64_t n, const int64_t *row_ptr, const int32_t *col,
                           const int64_t *w, const int32_t *c, const int64_t *delta,
                           int64_t tw, int64_t *degc /* scratch n */)
{
    int64_t inner = 0;
#pragma omp parallel for schedule(dynamic, 4096) reduction(+ : inner) num_threads(g_threads) if (g_threads > 1)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
            if (c[col[e]] == c[i])
                inner += w[e];
    memset(degc, 0, sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i)
        degc[c[i]] += delta[i];                      /* eq. 2 */
    i128 sq = 0;
    for (int64_t k = 0; k < n; ++k)
        sq += (i128)degc[k] * (i128)degc[k];
    return (i128)tw * (i128)inner - sq;
}

int orc_modularity(int64_t n, const int64_t *row_ptr, const int32_t *col, const int64_t *w,
                   const int32_t *labels, int64_t q_int[2], double *q)
{
    for (int64_t i = 0; i < n; ++i)
        if (labels[i] < 0 || labels[i] >= n)
            return ORC_EINVAL;
    int64_t *delta = malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    int64_t *degc = malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    if (!delta || !degc) { free(delta); free(degc); return ORC_ENOMEM; }
    int64_t tw;
    orc_degrees(n, row_ptr, w, delta, &tw);
    i128 v = modularity_int(n, row_ptr, col, w, labels, delta, tw, degc);
    put_i128(v, q_int);
    *q = tw ? (double)v / ((double)tw * (double)tw) : 0.0;
    free(delta);
    free(degc);
    return ORC_OK;
}

/* 64 x 128 -> 192-bit product, as (hi, lo). */
static void mul_u128_u64(u128 a, uint64_t b, uint64_t *hi, u128 *lo)
{
    u128 p0 = (u128)(uint64_t)a * b;
    u128 p1 = (u128)(uint64_t)(a >> 64) * b;
    u128 l = p0 + (p1 << 64);
    uint64_t carry = l < p0;
    *lo = l;
    *hi = (uint64_t)(p1 >> 64) + carry;
}

/* Keep a sweep iff theta_den * (q_new - q_prev) > theta_num * |q_prev|, with
 * theta = theta_num / theta_den the relative-gain threshold of Alg. 1. */
int orc_accept(const int64_t q_new[2], const int64_t q_prev[2], int64_t theta_num, int64_t theta_den)
{
    i128 qn = get_i128(q_new), qp = get_i128(q_prev);
    if (qn <= qp)
        return 0;
    u128 gain = (u128)(qn - qp);
    u128 mag = (u128)(qp < 0 ? -qp : qp);
    uint64_t lh, rh;
    u128 ll, rl;
    mul_u128_u64(gain, (uint64_t)theta_den, &lh, &ll);
    mul_u128_u64(mag, (uint64_t)theta_num, &rh, &rl);
    return lh > rh || (lh == rh && ll > rl);
}

/* One synchronous sweep (the parallel loop of Alg. 1).  Reads the snapshot
 * (c, degc, size) and writes every vertex's decision to c_out; e_self_out
 * (optional) gets e_{i->c_i} including i's loop.  acc (n per thread, zeroed)
 * and list (n per thread) are scratch. */
static void sweep(int64_t n, const int64_t *row_ptr, const int32_t *col, const int64_t *w,
                  const int64_t *delta, int64_t tw, const int32_t *c, const int64_t *degc,
                  const int32_t *size, int singlet_rule, int32_t *c_out, int64_t *e_self_out,
                  int64_t *acc_all, int32_t *list_all)
{
#pragma omp parallel for schedule(dynamic, 1024) num_threads(g_threads) if (g_threads > 1)
    for (int64_t i = 0; i < n; ++i) {
        int64_t *acc = acc_all + (size_t)THREAD_ID() * (size_t)n;
        int32_t *list = list_all + (size_t)THREAD_ID() * (size_t)n;
        int32_t ci = c[i];
        int64_t loop = 0;
        int64_t nl = 0;
        /* N_i: neighbouring communities and e_{i->C} (eq. 1), loops excluded */
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            int32_t j = col[e];
            if (j == i) { loop += w[e]; continue; }
            int32_t cj = c[j];
            if (acc[cj] == 0)
                list[nl++] = cj;
            acc[cj] += w[e];        /* weights >= 1, so acc > 0 once touched */
        }
        int64_t e_own = acc[ci];
        i128 s_own = (i128)tw * e_own - (i128)delta[i] * (i128)(degc[ci] - delta[i]);
        int32_t best = -1;
        i128 s_best = 0;
        for (int64_t k = 0; k < nl; ++k) {
            int32_t cand = list[k];
            if (cand == ci)
                continue;
            i128 s = (i128)tw * acc[cand] - (i128)delta[i] * (i128)degc[cand];
            if (best < 0 || s > s_best || (s == s_best && cand < best)) {
                best = cand;
                s_best = s;
            }
        }
        int32_t next = ci;
        if (best >= 0 && s_best > s_own) {
            if (singlet_rule && size[ci] == 1 && size[best] == 1 && best > ci)
                next = ci;               /* singlet minimum label heuristic */
            else
                next = best;
        }
        c_out[i] = next;
        if (e_self_out)
            e_self_out[i] = e_own + loop;
        for (int64_t k = 0; k < nl; ++k)
            acc[list[k]] = 0;
    }
}

/* The final merge (see the conventions above): from the snapshot (c, degc,
 * size), a vertex alone in its community whose neighbours other than
 * itself all carry one label C moves to C iff TW * e_{i->C} - delta_i *
 * deg_C beats its own score (zero for a vertex alone) and the singlet rule
 * allows it; every other vertex keeps its label.  Writes c_out. */
static void merge_one_neighbour(int64_t n, const int64_t *row_ptr, const int32_t *col, const int64_t *w,
                                const int64_t *delta, int64_t tw, const int32_t *c, const int64_t *degc,
                                const int32_t *size, int singlet_rule, int32_t *c_out)
{
    for (int64_t i = 0; i < n; ++i) {
        int32_t ci = c[i];
        c_out[i] = ci;
        if (size[ci] != 1)
            continue;
        int32_t target = -1;
        int single = 1;
        int64_t e_target = 0;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            int32_t j = col[e];
            if (j == i)
                continue;            /* loops take no part in moves */
            if (target < 0)
                target = c[j];
            else if (c[j] != target)
                single = 0;
            e_target += w[e];
        }
        if (target < 0 || !single)
            continue;
        /* i is alone, so e_{i->C(i)\{i}} = 0 and deg_{C(i)} - delta_i = 0 */
        i128 s_own = (i128)tw * 0 - (i128)delta[i] * (i128)(degc[ci] - delta[i]);
        i128 s = (i128)tw * e_target - (i128)delta[i] * (i128)degc[target];
        if (s <= s_own)
            continue;
        if (singlet_rule && size[target] == 1 && target > ci)
            continue;                /* singlet minimum label heuristic */
        c_out[i] = target;
    }
}

/* deg_C (eq. 2) and community sizes of labelling c. */
static void community_state(int64_t n, const int32_t *c, const int64_t *delta,
                            int64_t *degc, int32_t *size)
{
    memset(degc, 0, sizeof(int64_t) * (size_t)n);
    memset(size, 0, sizeof(int32_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        degc[c[i]] += delta[i];
        size[c[i]] += 1;
    }
}

/* One sweep from labels_in (NULL = singletons): labels_out, deg_C of the
 * new labelling (indexed by label), and e_{i->labels_in[i]} incl. loop. */
int orc_local_move(int64_t n, const int64_t *row_ptr, const int32_t *col, const int64_t *w,
                   const int32_t *labels_in, int singlet_rule, int32_t *labels_out,
                   int64_t *deg_out, int64_t *e_own_out)
{
    if (labels_in)
        for (int64_t i = 0; i < n; ++i)
            if (labels_in[i] < 0 || labels_in[i] >= n)
                return ORC_EINVAL;
    size_t nn = (size_t)(n ? n : 1);
    int64_t *delta = malloc(sizeof(int64_t) * nn), *degc = malloc(sizeof(int64_t) * nn);
    size_t nt = (size_t)g_threads;   /* scratch of the sweep: one row per thread */
    int64_t *acc = calloc(nn * nt, sizeof(int64_t));
    int32_t *size = malloc(sizeof(int32_t) * nn), *list = malloc(sizeof(int32_t) * nn * nt);
    int32_t *c = malloc(sizeof(int32_t) * nn);
    int rc = ORC_OK;
    if (!delta || !degc || !acc || !size || !list || !c) { rc = ORC_ENOMEM; goto out; }
    int64_t tw;
    orc_degrees(n, row_ptr, w, delta, &tw);
    for (int64_t i = 0; i < n; ++i)
        c[i] = labels_in ? labels_in[i] : (int32_t)i;
    community_state(n, c, delta, degc, size);
    sweep(n, row_ptr, col, w, delta, tw, c, degc, size, singlet_rule, labels_out, e_own_out, acc, list);
    if (deg_out) {
        community_state(n, labels_out, delta, degc, size);
        memcpy(deg_out, degc, sizeof(int64_t) * (size_t)n);
    }
out:
    free(delta); free(degc); free(acc); free(size); free(list); free(c);
    return rc;
}

/* The final merge alone, from labels_in (in [0, n)): labels_out. */
int orc_merge(int64_t n, const int64_t *row_ptr, const int32_t *col, const int64_t *w,
              const int32_t *labels_in, int singlet_rule, int32_t *labels_out)
{
    for (int64_t i = 0; i < n; ++i)
        if (labels_in[i] < 0 || labels_in[i] >= n)
            return ORC_EINVAL;
    size_t nn = (size_t)(n ? n : 1);
    int64_t *delta = malloc(sizeof(int64_t) * nn), *degc = malloc(sizeof(int64_t) * nn);
    int32_t *size = malloc(sizeof(int32_t) * nn);
    int rc = ORC_OK;
    if (!delta || !degc || !size) { rc = ORC_ENOMEM; goto out; }
    int64_t tw;
    orc_degrees(n, row_ptr, w, delta, &tw);
    community_state(n, labels_in, delta, degc, size);
    merge_one_neighbour(n, row_ptr, col, w, delta, tw, labels_in, degc, size, singlet_rule, labels_out);
out:
    free(delta); free(degc); free(size);
    return rc;
}

/* Renumbering: the new ID of label C is the number of distinct labels
 * smaller than C (consecutive IDs in ascending label order).  map has n
 * entries indexed by label; returns the number of communities. */
int64_t orc_renumber(int64_t n, const int32_t *c, int32_t *map)
{
    memset(map, 0, sizeof(int32_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i)
        map[c[i]] = 1;
    int64_t k = 0;
    for (int64_t v = 0; v < n; ++v) {
        int32_t present = map[v];
        map[v] = present ? (int32_t)k : -1;
        k += present;
    }
    return k;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Graph rebuilding: super-vertex a = {i : newc[i] = a}; A'_ab = sum of A_ij
 * over i in a, j in b.  Rows come out with ascending columns.  The output
 * arrays must hold n_new + 1 row pointers and nnz entries (contraction
 * never adds entries).  Returns nnz'. */
int64_t orc_contract(int64_t n, const int64_t *row_ptr, const int32_t *col, const int64_t *w,
                     const int32_t *newc, int64_t n_new, int64_t *rp_out, int32_t *col_out,
                     int64_t *w_out)
{
    size_t nn = (size_t)(n ? n : 1), nk = (size_t)(n_new ? n_new : 1);
    int64_t *start = calloc(nk + 1, sizeof(int64_t));
    int64_t *members = malloc(sizeof(int64_t) * nn);
    int64_t *fill = malloc(sizeof(int64_t) * nk);
    int64_t *acc = calloc(nk, sizeof(int64_t));
    int32_t *list = malloc(sizeof(int32_t) * nk);
    if (!start || !members || !fill || !acc || !list) {
        free(start); free(members); free(fill); free(acc); free(list);
        return -1;
    }
    for (int64_t i = 0; i < n; ++i)
        start[newc[i] + 1] += 1;
    for (int64_t a = 0; a < n_new; ++a)
        start[a + 1] += start[a];
    for (int64_t a = 0; a < n_new; ++a)
        fill[a] = start[a];
    for (int64_t i = 0; i < n; ++i)
        members[fill[newc[i]]++] = i;
    int64_t out = 0;
    rp_out[0] = 0;
    for (int64_t a = 0; a < n_new; ++a) {
        int64_t nl = 0;
        for (int64_t m = start[a]; m < start[a + 1]; ++m) {
            int64_t i = members[m];
            for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
                int32_t b = newc[col[e]];
                if (acc[b] == 0)
                    list[nl++] = b;
                acc[b] += w[e];
            }
        }
        qsort(list, (size_t)nl, sizeof(int32_t), cmp_i32);
        for (int64_t k = 0; k < nl; ++k) {
            col_out[out] = list[k];
            w_out[out] = acc[list[k]];
            acc[list[k]] = 0;
            ++out;
        }
        rp_out[a + 1] = out;
    }
    free(start); free(members); free(fill); free(acc); free(list);
    return out;
}

/* Per-level record of a run. */
typedef struct {
    int64_t n, nnz;
    int32_t sweeps_executed;   /* including the final discarded sweep */
    int32_t sweeps_accepted;
    int64_t q_int[2];          /* Q_int after the phase (on this level's graph) */
} orc_level_stats;

/*
 * The whole method (Alg. 2 driving Alg. 1 phases).
 *   w: int64 weights of the input graph.
 *   labels_out: final community of every input vertex, dense IDs.
 *   q_int/q: modularity of the final partition on the input graph.
 *   stats (optional): max_levels records; *levels_out: phases executed.
 * Returns ORC_OK, or ORC_ELIMIT if max_sweeps or max_levels cut the run
 * short (the result is still a valid partition).
 */
int orc_louvain(int64_t n, const int64_t *row_ptr, const int32_t *col, const int64_t *w,
                int64_t theta_num, int64_t theta_den, int32_t max_sweeps, int32_t max_levels,
                int singlet_rule, int merge, int32_t *labels_out, int64_t q_int[2], double *q,
                orc_level_stats *stats, int32_t *levels_out)
{
    size_t nn = (size_t)(n ? n : 1);
    int64_t nnz = row_ptr[n];
    size_t mm = (size_t)(nnz ? nnz : 1);
    int rc = ORC_OK;
    /* level graph (copied so that contraction can replace it) */
    int64_t *rp = malloc(sizeof(int64_t) * (nn + 1));
    int32_t *cl = malloc(sizeof(int32_t) * mm);
    int64_t *wt = malloc(sizeof(int64_t) * mm);
    int64_t *rp2 = malloc(sizeof(int64_t) * (nn + 1));
    int32_t *cl2 = malloc(sizeof(int32_t) * mm);
    int64_t *wt2 = malloc(sizeof(int64_t) * mm);
    int64_t *delta = malloc(sizeof(int64_t) * nn), *degc = malloc(sizeof(int64_t) * nn);
    int64_t *qscratch = malloc(sizeof(int64_t) * nn);
    size_t nt = (size_t)g_threads;   /* scratch of the sweep: one row per thread */
    int64_t *acc = calloc(nn * nt, sizeof(int64_t));
    int32_t *size = malloc(sizeof(int32_t) * nn), *list = malloc(sizeof(int32_t) * nn * nt);
    int32_t *c = malloc(sizeof(int32_t) * nn), *c_new = malloc(sizeof(int32_t) * nn);
    int32_t *map = malloc(sizeof(int32_t) * nn);
    if (!rp || !cl || !wt || !rp2 || !cl2 || !wt2 || !delta || !degc || !qscratch || !acc ||
        !size || !list || !c || !c_new || !map) {
        rc = ORC_ENOMEM;
        goto out;
    }
    memcpy(rp, row_ptr, sizeof(int64_t) * (size_t)(n + 1));
    memcpy(cl, col, sizeof(int32_t) * (size_t)nnz);
    memcpy(wt, w, sizeof(int64_t) * (size_t)nnz);
    for (int64_t v = 0; v < n; ++v)
        labels_out[v] = (int32_t)v;

    int64_t tw;
    orc_degrees(n, rp, wt, delta, &tw);
    i128 q_final = 0;
    int32_t levels = 0;
    int64_t ln = n;
    if (tw > 0)
        q_final = modularity_int(n, rp, cl, wt, labels_out, delta, tw, qscratch);
    while (tw > 0 && levels < max_levels) {
        /* initStatus: singleton communities */
        orc_degrees(ln, rp, wt, delta, &tw);
        for (int64_t i = 0; i < ln; ++i)
            c[i] = (int32_t)i;
        community_state(ln, c, delta, degc, size);
        i128 q_prev = modularity_int(ln, rp, cl, wt, c, delta, tw, qscratch);
        int32_t executed = 0, accepted = 0;
        /* Alg. 1: synchronous sweeps until the relative gain drops below theta */
        for (;;) {
            if (accepted >= max_sweeps) { rc = ORC_ELIMIT; break; }
            sweep(ln, rp, cl, wt, delta, tw, c, degc, size, singlet_rule, c_new, NULL, acc, list);
            ++executed;
            i128 q_new = modularity_int(ln, rp, cl, wt, c_new, delta, tw, qscratch);
            int64_t a[2], b[2];
            put_i128(q_new, a);
            put_i128(q_prev, b);
            if (!orc_accept(a, b, theta_num, theta_den))
                break;                       /* discard the sweep, end the phase */
            memcpy(c, c_new, sizeof(int32_t) * (size_t)ln);
            community_state(ln, c, delta, degc, size);
            q_prev = q_new;
            ++accepted;
        }
        if (merge && accepted > 0) {
            /* the final merge on the phase's labels, then Q once more */
            merge_one_neighbour(ln, rp, cl, wt, delta, tw, c, degc, size, singlet_rule, c_new);
            memcpy(c, c_new, sizeof(int32_t) * (size_t)ln);
            community_state(ln, c, delta, degc, size);
            q_prev = modularity_int(ln, rp, cl, wt, c, delta, tw, qscratch);
        }
        if (stats) {
            stats[levels].n = ln;
            stats[levels].nnz = rp[ln];
            stats[levels].sweeps_executed = executed;
            stats[levels].sweeps_accepted = accepted;
            put_i128(q_prev, stats[levels].q_int);
        }
        ++levels;
        if (accepted == 0)
            break;
        q_final = q_prev;
        /* renumber and compose the dendrogram level into the final labels */
        int64_t k = orc_renumber(ln, c, map);
        for (int64_t v = 0; v < n; ++v)
            labels_out[v] = map[c[labels_out[v]]];
        if (levels >= max_levels) { rc = ORC_ELIMIT; break; }
        /* induce the next level's graph */
        for (int64_t i = 0; i < ln; ++i)
            c_new[i] = map[c[i]];
        int64_t nnz2 = orc_contract(ln, rp, cl, wt, c_new, k, rp2, cl2, wt2);
        if (nnz2 < 0) { rc = ORC_ENOMEM; goto out; }
        int64_t *tp = rp; rp = rp2; rp2 = tp;
        int32_t *tc = cl; cl = cl2; cl2 = tc;
        int64_t *tw2 = wt; wt = wt2; wt2 = tw2;
        ln = k;
    }
    put_i128(q_final, q_int);
    orc_degrees(n, row_ptr, w, delta, &tw);
    *q = tw ? (double)q_final / ((double)tw * (double)tw) : 0.0;
    if (levels_out)
        *levels_out = levels;
out:
    free(rp); free(cl); free(wt); free(rp2); free(cl2); free(wt2);
    free(delta); free(degc); free(qscratch); free(acc); free(size); free(list);
    free(c); free(c_new); free(map);
    return rc;
}
