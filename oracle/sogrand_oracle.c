/*
 * SOGRAND reference oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, sequential CPU implementation of soft-output GRAND (SOGRAND)
 * list decoding of one component word and of block-turbo decoding of a 2-D
 * product code, written from the paper (Yuan, Medard, Galligan, Duffy,
 * "Soft-output (SO) GRAND and iterative decoding to outperform LDPCs",
 * arXiv 2310.10737).  Only the tests, the package smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or table with the GPU library.
 *
 * Precision: inputs and outputs are IEEE double; every probability is carried
 * in x86 80-bit long double.
 *
 * Readings of the paper taken here (the paper is silent or only cites):
 *  - Query order (ORBGRAND, cited in "Background on GRAND"): bits are ranked
 *    by |LLR| ascending (rank 1 = least reliable, ties broken by lower index);
 *    a pattern is a set of ranks; patterns are queried by logistic weight
 *    W = sum of ranks ascending, then Hamming weight ascending, then the rank
 *    tuple u_1<...<u_w in lexicographically ascending order.
 *  - Even codes (Sec. "Background on GRAND", parity argument): only patterns
 *    whose weight parity equals the parity of the hard decision are queried;
 *    skipped patterns are not counted as queries, and the query cap counts
 *    tested patterns only.
 *  - Soft output under the parity skip: Corollary 1 is applied inside the
 *    parity class -- the not-yet-queried mass is P(parity class) minus the
 *    queried mass, and the random-codebook hit probability is
 *    (2^k-1)/(2^(n-1)-1).  Codes that are not even use 1 - queried mass and
 *    (2^k-1)/(2^n-1).
 *  - When fewer than L codewords are found before the cap, the queried mass
 *    runs up to the last tested query (the list may even be empty).
 *  - The per-bit soft input in eq. (LLRi) is the SISO input L_Ch + L_A.
 *  - L_APP is clamped to [-1000, 1000] (reached only when a probability is
 *    exactly zero); a zero LLR decides bit 0.
 *  - List-BLER stop (the figures' "lists are added to until L or the predicted
 *    list-BLER is below tau"): after each codeword found before the L-th, the
 *    not-found probability of Corollary 1 is evaluated for the list so far, with
 *    the mass tested up to and including that codeword's query; the search ends
 *    when it is below tau (tau = 0: never).  The comparison is in binary64.
 *  - Product decoding (Sec. "Iterative decoding"): L_A = 0; half-iteration h
 *    decodes all rows (h odd) or all columns (h even) of L_Ch + L_A; the hard
 *    decision of L_APP is checked after every half-iteration (all rows and
 *    columns must be codewords); otherwise L_A = alpha L_E.  max_iter counts
 *    full row+column iterations.
 *  - QC-GLDPC codes (Sec. "Performance evaluation": the (n^2, n^2-2n(n-k))
 *    code whose adjacency matrix has the block rows [I(0) ... I(0)] and
 *    [I(0) I(1) ... I(n-1)], I(i) the n x n identity rotated right by i, so
 *    row r of I(i) has its one in column (r+i) mod n).  Variable node j*n + c
 *    is column c of block j; check node r of the first block row meets the
 *    variable nodes j*n + r, check node r of the second j*n + (r+j) mod n, and
 *    bit j of either component word is the one from block j.  The two block
 *    rows take the places of rows and columns in the block turbo loop above
 *    (first block row on odd h), each variable node taking its a-priori LLR
 *    from the other block row's last extrinsic output; validity requires every
 *    check node of both block rows.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ONMAX 256

/* ------------------------------------------------------------------------ */
/* query order: patterns of ranks in (W, w, lex) order                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n;
    long count, cap;      /* number stored, capacity */
    long max;             /* stop after this many patterns */
    int parity;           /* 0: even weights, 1: odd weights, -1: all */
    long *off;            /* pattern t occupies ranks[off[t] .. off[t+1]) */
    uint8_t *ranks;
    long nranks, rcap;
} oorder;

static void order_emit(oorder *o, const uint8_t *cur, int w) {
    if (o->count + 2 > o->cap) {
        o->cap = o->cap ? 2 * o->cap : 1024;
        o->off = (long *)realloc(o->off, (size_t)o->cap * sizeof(long));
    }
    if (o->nranks + w > o->rcap) {
        o->rcap = (o->rcap ? 2 * o->rcap : 4096) + w;
        o->ranks = (uint8_t *)realloc(o->ranks, (size_t)o->rcap);
    }
    o->off[o->count] = o->nranks;
    if (w > 0) memcpy(o->ranks + o->nranks, cur, (size_t)w);   /* the zero pattern stores nothing */
    o->nranks += w;
    o->count++;
    o->off[o->count] = o->nranks;
}

/* All strictly increasing tuples cur[pos..w-1] with parts in [lo, n] summing to rem,
   visited in lexicographically ascending order. */
static void order_rec(oorder *o, int pos, int w, int lo, long rem, uint8_t *cur) {
    if (o->count >= o->max) return;
    if (pos == w) {
        if (rem == 0) order_emit(o, cur, w);
        return;
    }
    int left = w - pos;
    for (int v = lo; v <= o->n; v++) {
        long minsum = (long)left * v + (long)left * (left - 1) / 2;
        if (minsum > rem) break;
        long maxsum = v + (long)(left - 1) * o->n - (long)(left - 1) * (left - 2) / 2;
        if (maxsum < rem) continue;
        cur[pos] = (uint8_t)v;
        order_rec(o, pos + 1, w, v + 1, rem - v, cur);
        if (o->count >= o->max) return;
    }
}

static void order_build(oorder *o, int n, int parity, long max) {
    memset(o, 0, sizeof(*o));
    o->n = n;
    o->parity = parity;
    o->max = max;
    o->off = (long *)malloc(sizeof(long));
    o->off[0] = 0;
    uint8_t cur[ONMAX];
    long wmaxsum = (long)n * (n + 1) / 2;
    for (long W = 0; W <= wmaxsum && o->count < max; W++) {
        for (int w = 0; w <= n && o->count < max; w++) {
            if (parity >= 0 && (w & 1) != parity) continue;
            long lo = (long)w * (w + 1) / 2;
            long hi = (long)w * n - (long)w * (w - 1) / 2;
            if (W < lo || W > hi) continue;
            order_rec(o, 0, w, 1, W, cur);
        }
    }
}

static void order_free(oorder *o) {
    free(o->off);
    free(o->ranks);
    memset(o, 0, sizeof(*o));
}

/* Exported for the order tests: the first max patterns of a class.
   ranks_out is [max][wcols] (zero padded), w_out is [max]; returns count
   (or -1 if a pattern is wider than wcols). */
long oracle_order(int n, int parity, long max, int wcols, uint8_t *ranks_out, uint8_t *w_out) {
    oorder o;
    if (n < 1 || n > ONMAX) return -2;
    order_build(&o, n, parity, max);
    long cnt = o.count;
    for (long t = 0; t < cnt; t++) {
        long w = o.off[t + 1] - o.off[t];
        if (w > wcols) { order_free(&o); return -1; }
        memset(ranks_out + t * wcols, 0, (size_t)wcols);
        memcpy(ranks_out + t * wcols, o.ranks + o.off[t], (size_t)w);
        w_out[t] = (uint8_t)w;
    }
    order_free(&o);
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* code                                                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n, k, r;
    uint64_t hcol[ONMAX];
    int even;
} ocode;

/* A linear code is even iff the all-ones word lies in the row space of H
   (the dual code).  Plain GF(2) elimination on rows stored as bit arrays. */
static int code_is_even(const ocode *c) {
    uint8_t rows[64 + 1][ONMAX];
    int nr = c->r;
    for (int r = 0; r < nr; r++)
        for (int j = 0; j < c->n; j++) rows[r][j] = (uint8_t)((c->hcol[j] >> r) & 1);
    uint8_t ones[ONMAX];
    for (int j = 0; j < c->n; j++) ones[j] = 1;
    int rank = 0;
    int pivcol[65];
    for (int col = 0; col < c->n && rank < nr; col++) {
        int sel = -1;
        for (int r = rank; r < nr; r++) if (rows[r][col]) { sel = r; break; }
        if (sel < 0) continue;
        if (sel != rank) {
            uint8_t tmp[ONMAX];
            memcpy(tmp, rows[sel], ONMAX); memcpy(rows[sel], rows[rank], ONMAX); memcpy(rows[rank], tmp, ONMAX);
        }
        for (int r = 0; r < nr; r++)
            if (r != rank && rows[r][col])
                for (int j = 0; j < c->n; j++) rows[r][j] ^= rows[rank][j];
        pivcol[rank] = col;
        rank++;
    }
    for (int r = 0; r < rank; r++)
        if (ones[pivcol[r]])
            for (int j = 0; j < c->n; j++) ones[j] ^= rows[r][j];
    for (int j = 0; j < c->n; j++) if (ones[j]) return 0;
    return 1;
}

static int code_init(ocode *c, int n, int k, const uint64_t *hcols) {
    if (n < 2 || n > ONMAX || k < 1 || k >= n || n - k > 64) return -1;
    c->n = n; c->k = k; c->r = n - k;
    for (int j = 0; j < n; j++) c->hcol[j] = hcols[j];
    c->even = code_is_even(c);
    return 0;
}

int oracle_code_is_even(int n, int k, const uint64_t *hcols) {
    ocode c;
    if (code_init(&c, n, k, hcols)) return -1;
    return c.even;
}

/* ------------------------------------------------------------------------ */
/* one component word                                                       */
/* ------------------------------------------------------------------------ */
typedef struct { double a; int i; } keyidx;

static int cmp_keyidx(const void *pa, const void *pb) {
    const keyidx *x = (const keyidx *)pa, *y = (const keyidx *)pb;
    if (x->a < y->a) return -1;
    if (x->a > y->a) return 1;
    return (x->i > y->i) - (x->i < y->i);
}

typedef struct {
    oorder ord[2];    /* even code: ord[parity]; other codes: ord[0] holds all weights */
    int even;
} oorders;

static void orders_build(oorders *os, const ocode *c, long qcap) {
    os->even = c->even;
    if (c->even) {
        order_build(&os->ord[0], c->n, 0, qcap);
        order_build(&os->ord[1], c->n, 1, qcap);
    } else {
        order_build(&os->ord[0], c->n, -1, qcap);
        memset(&os->ord[1], 0, sizeof(oorder));
    }
}

static void orders_free(oorders *os) {
    order_free(&os->ord[0]);
    if (os->even) order_free(&os->ord[1]);
}

typedef struct {
    /* outputs for one word; pointers may be NULL where noted */
    double *llr_app, *llr_ext;   /* [n] */
    uint8_t *hard;               /* [n] */
    uint32_t *n_queries;         /* [1] */
    int32_t *n_found;            /* [1] */
    uint32_t *found_q;           /* [L] */
    double *p_found;             /* [L] */
    double *p_notfound;          /* [1] */
    uint8_t *found_z;            /* [L][n] or NULL */
    double *diag;                /* [5] p0, queried mass, not-found mass, parity-class mass, and 1 if
                                    the class was exhausted (else 0); or NULL */
} oword_out;

typedef struct {
    keyidx *ki;
    int *perm;
    long double *rho;
    uint8_t *zlist;    /* [L][n] */
    long double *pz;   /* [L] */
} oscratch;

static void scratch_init(oscratch *s, int n, int L) {
    s->ki = (keyidx *)malloc(sizeof(keyidx) * n);
    s->perm = (int *)malloc(sizeof(int) * n);
    s->rho = (long double *)malloc(sizeof(long double) * n);
    s->zlist = (uint8_t *)malloc((size_t)L * n);
    s->pz = (long double *)malloc(sizeof(long double) * L);
}

static void scratch_free(oscratch *s) {
    free(s->ki); free(s->perm); free(s->rho); free(s->zlist); free(s->pz);
}

static void decode_word(const ocode *c, const oorders *os, const double *lam, int L, long qcap,
                        double pstop, oscratch *sc, const oword_out *out) {
    const int n = c->n;
    /* 1. hard decision: bit 1 iff the LLR log p(0)/p(1) is negative */
    uint8_t y[ONMAX];
    int ypar = 0;
    for (int i = 0; i < n; i++) { y[i] = lam[i] < 0.0; ypar ^= y[i]; }

    /* 2. reliability ranking: sort |lambda| ascending, ties by index */
    for (int i = 0; i < n; i++) { sc->ki[i].a = fabs(lam[i]); sc->ki[i].i = i; }
    qsort(sc->ki, (size_t)n, sizeof(keyidx), cmp_keyidx);
    for (int r = 0; r < n; r++) sc->perm[r] = sc->ki[r].i;   /* rank r+1 -> bit */

    /* 3. syndrome of the hard decision */
    uint64_t s0 = 0;
    for (int i = 0; i < n; i++) if (y[i]) s0 ^= c->hcol[i];

    /* 4. noise-effect probabilities: P(bit i flipped | r_i) = 1/(1+e^{a_i}); writing
          rho_i = e^{-a_i}, p(z|r) = p0 * prod_{i in z} rho_i with p0 = prod 1/(1+rho_i). */
    long double p0 = 1.0L;
    for (int i = 0; i < n; i++) {
        sc->rho[i] = expl(-(long double)fabs(lam[i]));
        p0 *= 1.0L / (1.0L + sc->rho[i]);
    }

    /* 5. mass of the hard decision's parity class (needed by Corollary 1, and by
          the list-BLER stop inside the loop).  It is p0 * (1[zero in class] + E or
          O), where E and O are the sums of prod rho over nonzero even / odd subsets,
          obtained by adding bits one at a time: E' = E + O rho_i, O' = O + (1 + E) rho_i. */
    const int zero_in_class = c->even ? (ypar == 0) : 1;
    long double E = 0.0L, O = 0.0L;
    for (int i = 0; i < n; i++) {
        long double e2 = E + O * sc->rho[i];
        long double o2 = O + (1.0L + E) * sc->rho[i];
        E = e2; O = o2;
    }
    const long double T_nz = c->even ? (ypar ? O : E) : (E + O);
    long double phi;
    if (c->even) phi = (ldexpl(1.0L, c->k) - 1.0L) / (ldexpl(1.0L, n - 1) - 1.0L);
    else         phi = (ldexpl(1.0L, c->k) - 1.0L) / (ldexpl(1.0L, n) - 1.0L);

    /* 6. GRAND query loop in ORBGRAND order, parity-matched for even codes.  It
          stops at the L-th codeword, at the cap, or (pstop > 0) as soon as the
          list-BLER predicted by Corollary 1 for the list so far, with the mass
          tested up to this codeword, is below pstop; that test is taken in binary64. */
    const oorder *ord = c->even ? &os->ord[ypar] : &os->ord[0];
    /* size of the queried class: every pattern of the hard decision's parity (even
       codes) or every pattern; 0 when it exceeds any query cap */
    const int cbits = c->even ? n - 1 : n;
    const long class_size = cbits <= 40 ? (1L << cbits) : 0;
    long t = 0;
    int stopped = 0;
    int found = 0;
    long double S_nz = 0.0L;   /* sum of p(z)/p0 over tested nonzero patterns */
    int zero_tested = 0;
    while (t < ord->count && t < qcap && found < L && !stopped) {
        const uint8_t *u = ord->ranks + ord->off[t];
        int w = (int)(ord->off[t + 1] - ord->off[t]);
        uint64_t s = s0;
        long double tau = 1.0L;
        for (int j = 0; j < w; j++) {
            int bit = sc->perm[u[j] - 1];
            s ^= c->hcol[bit];
            tau *= sc->rho[bit];
        }
        t++;
        if (w == 0) zero_tested = 1; else S_nz += tau;
        if (s == 0) {
            uint8_t *z = sc->zlist + (size_t)found * n;
            memset(z, 0, (size_t)n);
            for (int j = 0; j < w; j++) z[sc->perm[u[j] - 1]] = 1;
            sc->pz[found] = p0 * tau;
            if (out->found_q) out->found_q[found] = (uint32_t)t;
            found++;
            if (pstop > 0.0 && found < L) {
                long double Mi = p0 * ((long double)(zero_in_class - zero_tested) + (T_nz - S_nz));
                if (Mi < 0.0L || t == class_size) Mi = 0.0L;   /* nothing left untested */
                long double Di = Mi * phi;
                for (int l = 0; l < found; l++) Di += sc->pz[l];
                if ((double)((Mi * phi) / Di) < pstop) stopped = 1;
            }
        }
    }
    const long Q = t;

    /* 7. not-found mass and block soft output (Corollary 1).  Once every pattern of
          the class has been tested, the untested mass is exactly zero; the
          subtraction would leave only its rounding residue. */
    long double M = p0 * ((long double)(zero_in_class - zero_tested) + (T_nz - S_nz));
    if (M < 0.0L || Q == class_size) M = 0.0L;
    long double D = M * phi;
    for (int l = 0; l < found; l++) D += sc->pz[l];
    long double Pnf = (M * phi) / D;

    /* 8. bitwise soft output, eq. (LLRi), and the extrinsic LLR */
    for (int i = 0; i < n; i++) {
        long double N0 = 0.0L, N1 = 0.0L;
        for (int l = 0; l < found; l++) {
            long double P = sc->pz[l] / D;
            int ci = y[i] ^ sc->zlist[(size_t)l * n + i];
            if (ci) N1 += P; else N0 += P;
        }
        long double sig0 = 1.0L / (1.0L + expl(-(long double)lam[i]));   /* p(bit = 0 | SI) */
        long double sig1 = 1.0L / (1.0L + expl((long double)lam[i]));    /* p(bit = 1 | SI) */
        N0 += Pnf * sig0;
        N1 += Pnf * sig1;
        long double Lapp = logl(N0) - logl(N1);
        if (!(Lapp <= 1000.0L)) Lapp = 1000.0L;    /* +inf */
        if (!(Lapp >= -1000.0L)) Lapp = -1000.0L;  /* -inf */
        double la = (double)Lapp;
        if (out->llr_app) out->llr_app[i] = la;
        if (out->llr_ext) out->llr_ext[i] = la - lam[i];
        if (out->hard) out->hard[i] = la < 0.0;
    }
    if (out->n_queries) *out->n_queries = (uint32_t)Q;
    if (out->n_found) *out->n_found = found;
    if (out->p_found) for (int l = 0; l < found; l++) out->p_found[l] = (double)(sc->pz[l] / D);
    if (out->p_notfound) *out->p_notfound = (double)Pnf;
    if (out->found_z) memcpy(out->found_z, sc->zlist, (size_t)found * n);
    if (out->diag) {
        out->diag[0] = (double)p0;
        out->diag[1] = (double)(p0 * ((long double)zero_tested + S_nz));
        out->diag[2] = (double)M;
        out->diag[3] = (double)(p0 * ((long double)zero_in_class + T_nz));
        out->diag[4] = Q == class_size ? 1.0 : 0.0;
    }
}

/* Component decode of nwords independent words, row-major [nwords][n].
   found_q/p_found are [nwords][list_max]; entries past n_found are left zero.
   found_z ([nwords][list_max][n]) and diag ([nwords][5]) may be NULL. */
int oracle_decode_component(int n, int k, const uint64_t *hcols, long nwords, const double *llr,
                            int list_max, long qcap, double pstop,
                            double *llr_app, double *llr_ext, uint8_t *hard,
                            uint32_t *n_queries, int32_t *n_found, uint32_t *found_q,
                            double *p_found, double *p_notfound, uint8_t *found_z, double *diag) {
    ocode c;
    if (code_init(&c, n, k, hcols)) return -1;
    if (list_max < 1 || qcap < 1 || !(pstop >= 0.0 && pstop <= 1.0)) return -1;
    oorders os;
    orders_build(&os, &c, qcap);
    oscratch sc;
    scratch_init(&sc, n, list_max);
    for (long wd = 0; wd < nwords; wd++) {
        oword_out o;
        o.llr_app = llr_app + wd * n;
        o.llr_ext = llr_ext + wd * n;
        o.hard = hard + wd * n;
        o.n_queries = n_queries + wd;
        o.n_found = n_found + wd;
        o.found_q = found_q + wd * list_max;
        o.p_found = p_found + wd * list_max;
        o.p_notfound = p_notfound + wd;
        o.found_z = found_z ? found_z + (size_t)wd * list_max * n : NULL;
        o.diag = diag ? diag + wd * 5 : NULL;
        memset(o.found_q, 0, sizeof(uint32_t) * list_max);
        memset(o.p_found, 0, sizeof(double) * list_max);
        if (o.found_z) memset(o.found_z, 0, (size_t)list_max * n);
        decode_word(&c, &os, llr + wd * n, list_max, qcap, pstop, &sc, &o);
    }
    scratch_free(&sc);
    orders_free(&os);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* product codes and QC-GLDPC codes, block turbo decoding                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    const ocode *c;
    const oorders *os;
    int topo;    /* 0: product code, 1: QC-GLDPC */
    long nframes;
    const double *llr_ch;
    int list_max, max_iter, early_stop, store_f32;
    long qcap;
    double pstop;
    double alpha;
    uint8_t *hard;
    double *llr_app;
    uint8_t *success;
    uint16_t *half_iters;
    uint64_t *sum_q, *sum_maxq;
    double *last_diag;   /* [F][n][5] per word of the last half-iteration, or NULL */
    double *kappa_max;   /* [F] largest condition number of a not-found mass, or NULL */
    long next;   /* shared frame counter */
} oprod_job;

static int line_is_codeword(const ocode *c, const uint8_t *bits, long stride) {
    uint64_t s = 0;
    for (int j = 0; j < c->n; j++) if (bits[j * stride]) s ^= c->hcol[j];
    return s == 0;
}

/* Variable node (index into the frame) of bit j of component word `line` of
   family `fam` (0: rows / first block row, 1: columns / second block row). */
static long vnode(int topo, int n, int fam, int line, int j) {
    if (topo == 0) return fam == 0 ? (long)line * n + j : (long)j * n + line;
    return fam == 0 ? (long)j * n + line : (long)j * n + (line + j) % n;
}

int oracle_vnode(int topo, int n, int fam, int line, int j) {
    if (topo < 0 || topo > 1 || n < 1 || fam < 0 || fam > 1 || line < 0 || line >= n || j < 0 || j >= n)
        return -1;
    return (int)vnode(topo, n, fam, line, j);
}

/* every component word of both families of the hard decision C is a codeword */
static int frame_is_codeword(const ocode *c, int topo, const uint8_t *C) {
    const int n = c->n;
    uint8_t w[ONMAX];
    for (int fam = 0; fam < 2; fam++)
        for (int line = 0; line < n; line++) {
            for (int j = 0; j < n; j++) w[j] = C[vnode(topo, n, fam, line, j)];
            if (!line_is_codeword(c, w, 1)) return 0;
        }
    return 1;
}

static void decode_frame(const oprod_job *J, long f, oscratch *sc, double *LA, double *LE,
                         double *LAPP, uint8_t *C, double *lam, double *app, double *ext,
                         uint8_t *hd, uint32_t *fq, double *pf, double *dg) {
    const ocode *c = J->c;
    const int n = c->n;
    const double *Lch = J->llr_ch + (size_t)f * n * n;
    for (int i = 0; i < n * n; i++) LA[i] = 0.0;
    uint64_t sq = 0, smq = 0;
    int ok = 0, h;
    /* condition number of M = class mass - tested mass over every word decoded: the
       subtraction loses log2 of it in bits (0 when the class was exhausted, M = 0 exactly) */
    double kmax = 0.0;
    for (h = 1; h <= 2 * J->max_iter; h++) {
        const int fam = (h & 1) ? 0 : 1;   /* rows / first block row on odd h */
        uint32_t qmax = 0;
        for (int line = 0; line < n; line++) {
            for (int j = 0; j < n; j++) {
                long idx = vnode(J->topo, n, fam, line, j);
                lam[j] = Lch[idx] + LA[idx];
            }
            uint32_t q; int32_t nf; double pnf;
            oword_out o = { app, ext, hd, &q, &nf, fq, pf, &pnf, NULL, dg + (size_t)line * 5 };
            decode_word(c, J->os, lam, J->list_max, J->qcap, J->pstop, sc, &o);
            sq += q;
            if (q > qmax) qmax = q;
            {
                const double *d = dg + (size_t)line * 5;
                double kw = d[4] > 0.0 ? 0.0 : (d[2] > 0.0 ? d[3] / d[2] : INFINITY);
                if (kw > kmax) kmax = kw;
            }
            for (int j = 0; j < n; j++) {
                long idx = vnode(J->topo, n, fam, line, j);
                LAPP[idx] = app[j];
                LE[idx] = ext[j];
                C[idx] = hd[j];
            }
        }
        smq += qmax;
        const int valid = frame_is_codeword(c, J->topo, C);
        ok = valid;
        if ((valid && J->early_stop) || h == 2 * J->max_iter) break;
        for (int i = 0; i < n * n; i++) {
            double a = J->alpha * LE[i];
            LA[i] = J->store_f32 ? (double)(float)a : a;
        }
    }
    if (h > 2 * J->max_iter) h = 2 * J->max_iter;
    memcpy(J->hard + (size_t)f * n * n, C, (size_t)n * n);
    if (J->llr_app) memcpy(J->llr_app + (size_t)f * n * n, LAPP, sizeof(double) * n * n);
    if (J->last_diag) memcpy(J->last_diag + (size_t)f * n * 5, dg, sizeof(double) * n * 5);
    if (J->kappa_max) J->kappa_max[f] = kmax;
    J->success[f] = (uint8_t)ok;
    J->half_iters[f] = (uint16_t)h;
    J->sum_q[f] = sq;
    J->sum_maxq[f] = smq;
}

static void *prod_worker(void *arg) {
    oprod_job *J = (oprod_job *)arg;
    const int n = J->c->n;
    oscratch sc;
    scratch_init(&sc, n, J->list_max);
    double *LA = (double *)malloc(sizeof(double) * n * n);
    double *LE = (double *)malloc(sizeof(double) * n * n);
    double *LAPP = (double *)malloc(sizeof(double) * n * n);
    uint8_t *C = (uint8_t *)malloc((size_t)n * n);
    double *lam = (double *)malloc(sizeof(double) * n);
    double *app = (double *)malloc(sizeof(double) * n);
    double *ext = (double *)malloc(sizeof(double) * n);
    uint8_t *hd = (uint8_t *)malloc((size_t)n);
    uint32_t *fq = (uint32_t *)malloc(sizeof(uint32_t) * J->list_max);
    double *pf = (double *)malloc(sizeof(double) * J->list_max);
    double *dg = (double *)malloc(sizeof(double) * n * 5);
    for (;;) {
        long f = __atomic_fetch_add(&J->next, 1, __ATOMIC_RELAXED);
        if (f >= J->nframes) break;
        decode_frame(J, f, &sc, LA, LE, LAPP, C, lam, app, ext, hd, fq, pf, dg);
    }
    free(LA); free(LE); free(LAPP); free(C); free(lam); free(app); free(ext); free(hd); free(fq); free(pf);
    free(dg);
    scratch_free(&sc);
    return NULL;
}

/* Product decode of nframes frames [nframes][n][n] of channel LLRs.
   store_f32 != 0 stores the exchanged a-priori LLRs in binary32 (the caller
   passes binary32-representable channel LLRs).  llr_app may be NULL.  last_diag, if not
   NULL, receives [F][n][5]: the diag entries of each word of the frame's last
   half-iteration (word = row on odd, column on even half-iterations).  kappa_max, if
   not NULL, receives [F] the largest condition number class mass / not-found mass
   over every word the frame decoded (0 for an exhausted class, inf where the
   not-found mass vanished without exhaustion). */
static int decode_two_families(int topo, int n, int k, const uint64_t *hcols, long nframes,
                               const double *llr_ch, int list_max, long qcap, double pstop, int max_iter,
                               double alpha, int early_stop, int store_f32, uint8_t *hard, double *llr_app,
                               uint8_t *success, uint16_t *half_iters, uint64_t *sum_q, uint64_t *sum_maxq,
                               double *last_diag, double *kappa_max, int nthreads) {
    ocode c;
    if (code_init(&c, n, k, hcols)) return -1;
    if (list_max < 1 || qcap < 1 || max_iter < 1 || !(pstop >= 0.0 && pstop <= 1.0)) return -1;
    oorders os;
    orders_build(&os, &c, qcap);
    oprod_job J = { &c, &os, topo, nframes, llr_ch, list_max, max_iter, early_stop, store_f32, qcap, pstop,
                    alpha, hard, llr_app, success, half_iters, sum_q, sum_maxq, last_diag, kappa_max, 0 };
    if (nthreads < 1) nthreads = 1;
    if (nthreads == 1) {
        prod_worker(&J);
    } else {
        pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * nthreads);
        for (int t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, prod_worker, &J);
        for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
        free(th);
    }
    orders_free(&os);
    return 0;
}

/* Block turbo decoding of (n^2, k^2) product-code frames, row-major [F][n][n]. */
int oracle_decode_product(int n, int k, const uint64_t *hcols, long nframes, const double *llr_ch,
                          int list_max, long qcap, double pstop, int max_iter, double alpha, int early_stop,
                          int store_f32, uint8_t *hard, double *llr_app, uint8_t *success,
                          uint16_t *half_iters, uint64_t *sum_q, uint64_t *sum_maxq, double *last_diag, double *kappa_max,
                          int nthreads) {
    return decode_two_families(0, n, k, hcols, nframes, llr_ch, list_max, qcap, pstop, max_iter, alpha,
                               early_stop, store_f32, hard, llr_app, success, half_iters, sum_q, sum_maxq,
                               last_diag, kappa_max, nthreads);
}

/* The same loop over (n^2, n^2 - 2n(n-k)) QC-GLDPC frames, variable node j*n + c
   (column c of block j) at index j*n + c of [F][n*n]. */
int oracle_decode_gldpc(int n, int k, const uint64_t *hcols, long nframes, const double *llr_ch,
                        int list_max, long qcap, double pstop, int max_iter, double alpha, int early_stop,
                        int store_f32, uint8_t *hard, double *llr_app, uint8_t *success,
                        uint16_t *half_iters, uint64_t *sum_q, uint64_t *sum_maxq, double *last_diag, double *kappa_max,
                          int nthreads) {
    return decode_two_families(1, n, k, hcols, nframes, llr_ch, list_max, qcap, pstop, max_iter, alpha,
                               early_stop, store_f32, hard, llr_app, success, half_iters, sum_q, sum_maxq,
                               last_diag, kappa_max, nthreads);
}
