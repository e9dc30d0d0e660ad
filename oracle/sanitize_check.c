/* Test infrastructure only: runs the oracle's component, product and QC-GLDPC entry points
 * on inputs read from a file and writes their outputs to another, so that the oracle can be
 * built with the address and undefined-behaviour sanitizers and its results compared with
 * those of the regular build.
 *
 * Input (native byte order): int32 n, k, list_max, max_iter, nthreads; int64 qcap, nwords,
 * nframes; double pstop, alpha; uint64 hcols[n]; double words[nwords][n];
 * double product_frames[nframes][n][n]; double gldpc_frames[nframes][n][n].
 * Output: for the words, llr_app, llr_ext, hard, n_queries, n_found, found_q, p_found,
 * p_notfound; for each of the two frame sets, hard, llr_app, success, half_iters, sum_q,
 * sum_maxq, kappa_max.  Exit status 0 on success.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_decode_component(int n, int k, const uint64_t *hcols, long nwords, const double *llr,
                            int list_max, long qcap, double pstop,
                            double *llr_app, double *llr_ext, uint8_t *hard,
                            uint32_t *n_queries, int32_t *n_found, uint32_t *found_q,
                            double *p_found, double *p_notfound, uint8_t *found_z, double *diag);
int oracle_decode_product(int n, int k, const uint64_t *hcols, long nframes, const double *llr_ch,
                          int list_max, long qcap, double pstop, int max_iter, double alpha, int early_stop,
                          int store_f32, uint8_t *hard, double *llr_app, uint8_t *success,
                          uint16_t *half_iters, uint64_t *sum_q, uint64_t *sum_maxq, double *last_diag,
                          double *kappa_max, int nthreads);
int oracle_decode_gldpc(int n, int k, const uint64_t *hcols, long nframes, const double *llr_ch,
                        int list_max, long qcap, double pstop, int max_iter, double alpha, int early_stop,
                        int store_f32, uint8_t *hard, double *llr_app, uint8_t *success,
                        uint16_t *half_iters, uint64_t *sum_q, uint64_t *sum_maxq, double *last_diag,
                        double *kappa_max, int nthreads);

static void *take(FILE *f, size_t bytes) {
    void *p = malloc(bytes ? bytes : 1);
    if (!p || fread(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "short input\n");
        exit(2);
    }
    return p;
}

static void put(FILE *f, const void *p, size_t bytes) {
    if (fwrite(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "short write\n");
        exit(2);
    }
}

static int frames(FILE *out, int gldpc, int n, int k, const uint64_t *h, long F, const double *llr, int L, long qcap,
                  double pstop, int iters, double alpha, int nthreads) {
    const size_t nn = (size_t)n * n;
    uint8_t *hard = calloc(F * nn, 1), *succ = calloc(F, 1);
    double *app = calloc(F * nn, sizeof(double)), *kap = calloc(F, sizeof(double));
    uint16_t *hi = calloc(F, sizeof(uint16_t));
    uint64_t *sq = calloc(F, sizeof(uint64_t)), *sm = calloc(F, sizeof(uint64_t));
    const int rc = (gldpc ? oracle_decode_gldpc : oracle_decode_product)(n, k, h, F, llr, L, qcap, pstop, iters,
                                                                         alpha, 1, 0, hard, app, succ, hi, sq, sm,
                                                                         NULL, kap, nthreads);
    put(out, hard, F * nn);
    put(out, app, F * nn * sizeof(double));
    put(out, succ, F);
    put(out, hi, F * sizeof(uint16_t));
    put(out, sq, F * sizeof(uint64_t));
    put(out, sm, F * sizeof(uint64_t));
    put(out, kap, F * sizeof(double));
    free(hard); free(succ); free(app); free(kap); free(hi); free(sq); free(sm);
    return rc;
}

int main(int argc, char **argv) {
    if (argc != 3) {
        fprintf(stderr, "usage: %s input output\n", argv[0]);
        return 2;
    }
    FILE *in = fopen(argv[1], "rb"), *out = fopen(argv[2], "wb");
    if (!in || !out) {
        fprintf(stderr, "cannot open files\n");
        return 2;
    }
    int32_t *hd = take(in, 5 * sizeof(int32_t));
    int64_t *sz = take(in, 3 * sizeof(int64_t));
    double *pr = take(in, 2 * sizeof(double));
    const int n = hd[0], k = hd[1], L = hd[2], iters = hd[3], nthreads = hd[4];
    const long qcap = (long)sz[0], W = (long)sz[1], F = (long)sz[2];
    uint64_t *h = take(in, (size_t)n * sizeof(uint64_t));
    double *words = take(in, (size_t)W * n * sizeof(double));
    double *pf = take(in, (size_t)F * n * n * sizeof(double));
    double *gf = take(in, (size_t)F * n * n * sizeof(double));
    fclose(in);

    double *app = calloc((size_t)W * n, sizeof(double)), *ext = calloc((size_t)W * n, sizeof(double));
    uint8_t *hard = calloc((size_t)W * n, 1);
    uint32_t *nq = calloc(W, sizeof(uint32_t)), *fq = calloc((size_t)W * L, sizeof(uint32_t));
    int32_t *nf = calloc(W, sizeof(int32_t));
    double *pf_l = calloc((size_t)W * L, sizeof(double)), *pnf = calloc(W, sizeof(double));
    int rc = oracle_decode_component(n, k, h, W, words, L, qcap, pr[0], app, ext, hard, nq, nf, fq, pf_l, pnf,
                                     NULL, NULL);
    put(out, app, (size_t)W * n * sizeof(double));
    put(out, ext, (size_t)W * n * sizeof(double));
    put(out, hard, (size_t)W * n);
    put(out, nq, W * sizeof(uint32_t));
    put(out, nf, W * sizeof(int32_t));
    put(out, fq, (size_t)W * L * sizeof(uint32_t));
    put(out, pf_l, (size_t)W * L * sizeof(double));
    put(out, pnf, W * sizeof(double));
    rc |= frames(out, 0, n, k, h, F, pf, L, qcap, pr[0], iters, pr[1], nthreads);
    rc |= frames(out, 1, n, k, h, F, gf, L, qcap, pr[0], iters, pr[1], nthreads);
    fclose(out);
    free(app); free(ext); free(hard); free(nq); free(fq); free(nf); free(pf_l); free(pnf);
    free(hd); free(sz); free(pr); free(h); free(words); free(pf); free(gf);
    return rc ? 1 : 0;
}
