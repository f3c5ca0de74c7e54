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
 * ORACLE_MUTANT (compile-time, default 0) plants one deliberate mistake so the
 * test suite can show that its pins catch it; products never set it.
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
