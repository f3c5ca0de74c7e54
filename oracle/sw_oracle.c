/*
 * CPU oracle for score-only Smith-Waterman with Gotoh affine gaps.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load or call this code.  It shares nothing
 * with the GPU library: no header, helper, table or layout code.
 *
 * What it computes (paper, Section 2.2, Eqs. for H, E and F):
 *
 *   H[i][j] = max(0, H[i-1][j-1] + SM(Q[i], D[j]), E[i][j], F[i][j])
 *   E[i][j] = max(H[i][j-1] - Go, E[i][j-1] - Ge)      (left neighbour)
 *   F[i][j] = max(H[i-1][j] - Go, F[i-1][j] - Ge)      (upper neighbour)
 *
 * with H, E and F equal to 0 on row i = 0 and column j = 0, for 1 <= i <= m
 * (query) and 1 <= j <= n (subject).  The result S is the largest H of the
 * matrix, which is the optimal local alignment score.  SM is the 32x32 int32
 * substitution matrix indexed [query residue][subject residue]; Go and Ge are
 * the non-negative magnitudes subtracted in the E and F equations.
 *
 * All arithmetic is int64 and plain scalar C: two rows of H and F (previous
 * and current) are kept, E runs along the current row.  Nothing is blocked,
 * fused or reordered beyond that.
 *
 * swo_align (below) adds the alignment itself for one pair.
 *
 * ORACLE_MUTANT (compile-time, default 0) plants one deliberate mistake so the
 * test suite can show that its pins catch it (1-7 in the score, 8-11 in the
 * traceback); products never set it.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

static int64_t max2(int64_t a, int64_t b) { return a > b ? a : b; }

/* One pair: the literal recurrence.  Returns S, or -1 when memory runs out. */
int64_t swo_score(const uint8_t *Q, int64_t m, const uint8_t *D, int64_t n,
                  const int32_t *SM, int64_t Go, int64_t Ge)
{
    if (m <= 0 || n <= 0)
        return 0;                       /* empty matrix: S = 0 */
    int64_t *Hprev = calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *Fprev = calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *Hcur = calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *Fcur = calloc((size_t)n + 1, sizeof(int64_t));
    if (!Hprev || !Fprev || !Hcur || !Fcur) {
        free(Hprev); free(Fprev); free(Hcur); free(Fcur);
        return -1;
    }
    int64_t S = 0;
    for (int64_t i = 1; i <= m; ++i) {
        Hcur[0] = 0;                    /* column j = 0 */
        Fcur[0] = 0;
        int64_t Eleft = 0;              /* E[i][0] = 0 */
        for (int64_t j = 1; j <= n; ++j) {
#if ORACLE_MUTANT == 3
            int64_t sm = SM[(int)D[j - 1] * 32 + (int)Q[i - 1]];   /* transposed */
#else
            int64_t sm = SM[(int)Q[i - 1] * 32 + (int)D[j - 1]];
#endif
#if ORACLE_MUTANT == 5
            int64_t E = max2(Hcur[j - 1] - Go - Ge, Eleft - Ge);   /* BLAST-style open */
#else
            int64_t E = max2(Hcur[j - 1] - Go, Eleft - Ge);
#endif
#if ORACLE_MUTANT == 2
            int64_t F = max2(Hprev[j] + Go, Fprev[j] - Ge);        /* sign slip */
#else
            int64_t F = max2(Hprev[j] - Go, Fprev[j] - Ge);
#endif
#if ORACLE_MUTANT == 4
            int64_t diag = Hprev[j];                                 /* wrong neighbour */
#else
            int64_t diag = Hprev[j - 1];
#endif
#if ORACLE_MUTANT == 1
            int64_t H = max2(max2(0, diag + sm), F);                 /* E dropped */
#elif ORACLE_MUTANT == 6
            int64_t H = max2(max2(diag + sm, E), F);                 /* no zero floor */
#else
            int64_t H = max2(max2(0, diag + sm), max2(E, F));
#endif
            Hcur[j] = H;
            Fcur[j] = F;
            Eleft = E;
#if ORACLE_MUTANT == 7
            if (i == m) S = max2(S, H);                              /* last row only */
#else
            S = max2(S, H);
#endif
        }
        int64_t *t = Hprev; Hprev = Hcur; Hcur = t;
        t = Fprev; Fprev = Fcur; Fcur = t;
    }
    free(Hprev); free(Fprev); free(Hcur); free(Fcur);
    return S;
}

/* ---------------------------------------------------------------- threads  */

struct job {
    const uint8_t *Q; int64_t m;
    const uint8_t *res; const int64_t *off; const int32_t *len;
    const int64_t *ids; int64_t nids;           /* subjects to score */
    const int32_t *SM; int64_t Go, Ge;
    int64_t *out;                               /* out[k] for ids[k] */
    int64_t next;                               /* shared work counter */
    int64_t chunk;
    int failed;
};

static void *worker(void *arg)
{
    struct job *jb = arg;
    for (;;) {
        int64_t k0 = __atomic_fetch_add(&jb->next, jb->chunk, __ATOMIC_RELAXED);
        if (k0 >= jb->nids)
            break;
        int64_t k1 = k0 + jb->chunk < jb->nids ? k0 + jb->chunk : jb->nids;
        for (int64_t k = k0; k < k1; ++k) {
            int64_t s = jb->ids ? jb->ids[k] : k;
            int64_t v = swo_score(jb->Q, jb->m, jb->res + jb->off[s], jb->len[s],
                                  jb->SM, jb->Go, jb->Ge);
            if (v < 0)
                __atomic_store_n(&jb->failed, 1, __ATOMIC_RELAXED);
            jb->out[k] = v;
        }
    }
    return NULL;
}

/*
 * Score one query against the subjects listed in ids[0..nids) (all nseq
 * subjects when ids is NULL and nids == nseq), on nthreads threads that take
 * subjects in dynamic chunks.  Returns 0, or -1 if a score could not be
 * computed (out of memory) or a thread could not be started.
 */
int swo_search(const uint8_t *Q, int64_t m, const uint8_t *res, const int64_t *off,
               const int32_t *len, const int64_t *ids, int64_t nids,
               const int32_t *SM, int64_t Go, int64_t Ge, int64_t *out, int nthreads)
{
    struct job jb;
    memset(&jb, 0, sizeof jb);
    jb.Q = Q; jb.m = m; jb.res = res; jb.off = off; jb.len = len;
    jb.ids = ids; jb.nids = nids; jb.SM = SM; jb.Go = Go; jb.Ge = Ge;
    jb.out = out; jb.chunk = 16;
    if (nthreads < 1)
        nthreads = 1;
    pthread_t *th = calloc((size_t)nthreads, sizeof(pthread_t));
    if (!th)
        return -1;
    int started = 0;
    for (int t = 0; t < nthreads; ++t) {
        if (pthread_create(&th[t], NULL, worker, &jb) != 0)
            break;
        ++started;
    }
    if (started == 0)
        worker(&jb);
    for (int t = 0; t < started; ++t)
        pthread_join(th[t], NULL);
    free(th);
    return jb.failed ? -1 : 0;
}

/*
 * One pair with its alignment (the traceback the paper mentions as the
 * optional step after the score, Section 2.2).  Full int64 matrices H, E, F of
 * (m+1) x (n+1) entries, filled with the same recurrence as swo_score.
 *
 * Reading of the unspecified choices (the paper gives none):
 *   end cell   the first cell with H = S in column-major order: smallest
 *              subject position j, then smallest query position i;
 *   traceback  from the end cell in state H: the diagonal term if it gives
 *              H, else E, else F; a gap state opens (from H) rather than
 *              extends when both give its value; the alignment begins at the
 *              diagonal step whose predecessor cell holds H = 0 (or lies on
 *              the border).
 * Output: S, 1-based inclusive begin/end positions, and the operations from
 * begin to end: 'M' (query residue aligned to subject residue), 'I' (query
 * residue against a gap, the F direction), 'D' (subject residue against a gap,
 * the E direction).  S = 0 gives an empty alignment (positions 0).
 * Returns the number of operations, -1 when memory runs out, -2 when `cap` is
 * too small.
 */
int64_t swo_align(const uint8_t *Q, int64_t m, const uint8_t *D, int64_t n, const int32_t *SM,
                  int64_t Go, int64_t Ge, int64_t *out5, char *ops, int64_t cap)
{
    out5[0] = out5[1] = out5[2] = out5[3] = out5[4] = 0;
    if (m <= 0 || n <= 0)
        return 0;
    const int64_t W = n + 1;
    const size_t cells = (size_t)(m + 1) * (size_t)W;
    int64_t *H = calloc(cells, sizeof(int64_t));
    int64_t *E = calloc(cells, sizeof(int64_t));
    int64_t *F = calloc(cells, sizeof(int64_t));
    if (!H || !E || !F) {
        free(H); free(E); free(F);
        return -1;
    }
#define AT(X, i, j) X[(size_t)(i) * (size_t)W + (size_t)(j)]
    for (int64_t i = 1; i <= m; ++i) {
        for (int64_t j = 1; j <= n; ++j) {
            const int64_t sm = SM[(int)Q[i - 1] * 32 + (int)D[j - 1]];
            AT(E, i, j) = max2(AT(H, i, j - 1) - Go, AT(E, i, j - 1) - Ge);
            AT(F, i, j) = max2(AT(H, i - 1, j) - Go, AT(F, i - 1, j) - Ge);
            AT(H, i, j) = max2(max2(0, AT(H, i - 1, j - 1) + sm), max2(AT(E, i, j), AT(F, i, j)));
        }
    }
    int64_t S = 0, bi = 0, bj = 0;
#if ORACLE_MUTANT == 8
    for (int64_t i = 1; i <= m; ++i)            /* row-major first maximum */
        for (int64_t j = 1; j <= n; ++j)
#else
    for (int64_t j = 1; j <= n; ++j)            /* column-major: first maximum */
        for (int64_t i = 1; i <= m; ++i)
#endif
            if (AT(H, i, j) > S) {
                S = AT(H, i, j);
                bi = i;
                bj = j;
            }
    int64_t nops = 0;
    if (S > 0) {
        int64_t i = bi, j = bj;
        int state = 0;                           /* 0: H, 1: E, 2: F */
        for (;;) {
            if (nops >= cap || i < 1 || j < 1) {  /* never reached by the rules above */
                free(H); free(E); free(F);
                return -2;
            }
            if (state == 0) {
                const int64_t sm = SM[(int)Q[i - 1] * 32 + (int)D[j - 1]];
                const int64_t h = AT(H, i, j);
#if ORACLE_MUTANT == 9
                if (h == AT(E, i, j)) {          /* gap before diagonal */
                    state = 1;
                } else if (h == AT(H, i - 1, j - 1) + sm) {
#else
                if (h == AT(H, i - 1, j - 1) + sm) {
#endif
                    ops[nops++] = 'M';
#if ORACLE_MUTANT == 11
                    if (i == 1 || j == 1)        /* runs on through H = 0 */
#else
                    if (i == 1 || j == 1 || AT(H, i - 1, j - 1) == 0)
#endif
                        break;                   /* begins here */
                    --i;
                    --j;
#if ORACLE_MUTANT == 9
                } else {
                    state = 2;
                }
#else
                } else if (h == AT(E, i, j)) {
                    state = 1;
                } else {
                    state = 2;
                }
#endif
            } else if (state == 1) {             /* E: subject residue j against a gap */
                ops[nops++] = 'D';
#if ORACLE_MUTANT == 10
                if (AT(E, i, j) != AT(E, i, j - 1) - Ge)    /* extend before open */
#else
                if (AT(E, i, j) == AT(H, i, j - 1) - Go)
#endif
                    state = 0;
                --j;
            } else {                             /* F: query residue i against a gap */
                ops[nops++] = 'I';
                if (AT(F, i, j) == AT(H, i - 1, j) - Go)
                    state = 0;
                --i;
            }
        }
        out5[1] = i;                             /* begin (query, subject) */
        out5[2] = j;
        for (int64_t a = 0, b = nops - 1; a < b; ++a, --b) {
            const char t = ops[a];
            ops[a] = ops[b];
            ops[b] = t;
        }
    }
#undef AT
    out5[0] = S;
    out5[3] = bi;                                /* end (query, subject) */
    out5[4] = bj;
    free(H); free(E); free(F);
    return nops;
}
