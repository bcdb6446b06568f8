/*
 * Test driver for a sanitizer build of the CPU oracle (AddressSanitizer and
 * UndefinedBehaviorSanitizer, host code only): reads graphs written by
 * tests/test_sanitize_cpu.py, runs the oracle's entry points on each (the
 * whole method with and without the final merge, one sweep, eq. 3,
 * renumbering and contraction, on one and on several OpenMP threads) and
 * writes their results for the test to compare with the regular build.
 *
 * Input file:  int64 n, int64 nnz, int64 row_ptr[n+1], int32 col[nnz],
 *              int64 w[nnz], int32 labels[n] (a labelling for the sweep,
 *              eq. 3 and the contraction).
 * Output file: for threads in {1, 3}: run labels[n], run q_int[2], merged
 *              run labels[n], merged q_int[2], sweep labels[n], sweep
 *              deg[n], sweep e_own[n], eq. 3 q_int[2], n_new, contracted
 *              row_ptr[n_new+1], col[nnz'], w[nnz'] (int64 n_new and nnz'
 *              first).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int64_t n, nnz;
    int32_t sweeps_executed, sweeps_accepted;
    int64_t q_int[2];
} orc_level_stats;

void orc_set_threads(int threads);
int orc_modularity(int64_t n, const int64_t *row_ptr, const int32_t *col, const int64_t *w, const int32_t *c,
                   int64_t q_int[2], double *q);
int orc_local_move(int64_t n, const int64_t *row_ptr, const int32_t *col, const int64_t *w, const int32_t *c_in,
                   int singlet_rule, int32_t *c_out, int64_t *deg_out, int64_t *e_own_out);
int64_t orc_renumber(int64_t n, const int32_t *c, int32_t *map);
int64_t orc_contract(int64_t n, const int64_t *row_ptr, const int32_t *col, const int64_t *w, const int32_t *map,
                     int64_t n_new, int64_t *rp_out, int32_t *col_out, int64_t *w_out);
int orc_louvain(int64_t n, const int64_t *row_ptr, const int32_t *col, const int64_t *w, int64_t theta_num,
                int64_t theta_den, int32_t max_sweeps, int32_t max_levels, int singlet_rule, int merge,
                int32_t *labels_out, int64_t q_int[2], double *q, orc_level_stats *stats, int32_t *levels_out);

static void *xread(FILE *f, size_t size, size_t count) {
    void *p = malloc(size * (count ? count : 1));
    if (!p || fread(p, size, count, f) != count) {
        fprintf(stderr, "short read\n");
        exit(2);
    }
    return p;
}

int main(int argc, char **argv) {
    if (argc != 3) {
        fprintf(stderr, "usage: %s graph.bin out.bin\n", argv[0]);
        return 2;
    }
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t n, nnz;
    if (fread(&n, 8, 1, f) != 1 || fread(&nnz, 8, 1, f) != 1) return 2;
    int64_t *rp = xread(f, 8, (size_t)n + 1);
    int32_t *col = xread(f, 4, (size_t)nnz);
    int64_t *w = xread(f, 8, (size_t)nnz);
    int32_t *lab = xread(f, 4, (size_t)n);
    fclose(f);
    FILE *o = fopen(argv[2], "wb");
    if (!o) return 2;
    const size_t nn = (size_t)(n ? n : 1), mm = (size_t)(nnz ? nnz : 1);
    int32_t *out = malloc(4 * nn), *map = malloc(4 * nn), *col2 = malloc(4 * mm);
    int64_t *deg = malloc(8 * nn), *eown = malloc(8 * nn), *rp2 = malloc(8 * (nn + 1)), *w2 = malloc(8 * mm);
    orc_level_stats st[64];
    int32_t levels = 0;
    int64_t q2[2];
    double q;
    const int threads[2] = {1, 3};
    for (int t = 0; t < 2; ++t) {
        orc_set_threads(threads[t]);
        for (int merge = 0; merge < 2; ++merge) {
            if (orc_louvain(n, rp, col, w, 1, 1000000, 1000, 64, 1, merge, out, q2, &q, st, &levels) < -1) return 3;
            fwrite(out, 4, (size_t)n, o);
            fwrite(q2, 8, 2, o);
        }
        if (orc_local_move(n, rp, col, w, lab, 1, out, deg, eown) != 0) return 3;
        fwrite(out, 4, (size_t)n, o);
        fwrite(deg, 8, (size_t)n, o);
        fwrite(eown, 8, (size_t)n, o);
        if (orc_modularity(n, rp, col, w, lab, q2, &q) != 0) return 3;
        fwrite(q2, 8, 2, o);
        const int64_t k = orc_renumber(n, lab, map);
        int32_t *newlab = malloc(4 * nn);
        for (int64_t i = 0; i < n; ++i) newlab[i] = map[lab[i]];
        const int64_t m2 = orc_contract(n, rp, col, w, newlab, k, rp2, col2, w2);
        free(newlab);
        fwrite(&k, 8, 1, o);
        fwrite(&m2, 8, 1, o);
        fwrite(rp2, 8, (size_t)k + 1, o);
        fwrite(col2, 4, (size_t)m2, o);
        fwrite(w2, 8, (size_t)m2, o);
    }
    fclose(o);
    free(rp); free(col); free(w); free(lab); free(out); free(map); free(col2);
    free(deg); free(eown); free(rp2); free(w2);
    return 0;
}
