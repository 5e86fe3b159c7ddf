/*
 * CPU oracle for batched global pairwise alignment.  TEST INFRASTRUCTURE ONLY:
 * the tests, the smoke check and the CPU-baseline leg of the benchmark call
 * it; the GPU library never does, and the two share no code.
 *
 * What it computes (paper: System and Methods, "Supported Alignment
 * Algorithms"): the optimal global alignment cost of a pattern P (length m)
 * against a text T (length n) and one optimal alignment as a CIGAR.
 *
 *   Needleman-Wunsch, linear gaps (NW subsection): one DP table H over m x n,
 *     H(i,j) = min(H(i-1,j-1) + c(i,j), H(i-1,j) + g, H(i,j-1) + g),
 *     H(i,0) = i g, H(0,j) = j g, c(i,j) = 0 if P_i = T_j else x.
 *   Smith-Waterman-Gotoh, affine gaps (SWG subsection): three tables,
 *     E(i,j) = min(H(i-1,j) + o + e, E(i-1,j) + e)      (gap in T: P_i alone)
 *     F(i,j) = min(H(i,j-1) + o + e, F(i,j-1) + e)      (gap in P: T_j alone)
 *     H(i,j) = min(H(i-1,j-1) + c(i,j), E(i,j), F(i,j))
 *     H(0,0) = 0, H(i,0) = E(i,0) = o + i e, F(i,0) = inf,
 *     H(0,j) = F(0,j) = o + j e, E(0,j) = inf.
 *   The wavefront algorithm (WFA subsection) reaches the same optimum as
 *   Gotoh, so the oracle for it is this Gotoh definition.
 *
 * A gap run of length L costs o + L e (the form in which one gap base costs
 * o + e, as in the WFA recurrences); match cost is 0, all costs minimised.
 *
 * Canonical traceback (the paper does not fix a tie-break; this is the
 * library's documented choice).  Walk back from (m,n) in state H and take the
 * first feasible candidate of:
 *   state H:  X  if P_i != T_j and H(i,j) = H(i-1,j-1) + x  -> (i-1,j-1), H
 *             I  if H(i,j) = E(i,j)                         -> state E
 *             D  if H(i,j) = F(i,j)                         -> state F
 *             =  if P_i == T_j and H(i,j) = H(i-1,j-1)      -> (i-1,j-1), H
 *   state E:  emit I; go to H at (i-1,j) if E(i,j) = H(i-1,j) + o + e (close
 *             the run here), else stay in E at (i-1,j).
 *   state F:  emit D; symmetric in j.
 *   NW: single state, order X, I (H = H(i-1,j) + g), D (H = H(i,j-1) + g), =.
 * Ops: '=' match, 'X' mismatch, 'I' consumes P only, 'D' consumes T only.
 *
 * Threshold: with max_score >= 0 a pair whose optimum exceeds max_score is
 * REJECTED (status 1, score -1, no CIGAR).
 *
 * CIGAR runs are uint32 (length << 4 | op) with op 0 '=', 1 'X', 2 'I', 3 'D'.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define INF (INT32_MAX / 2)
enum { OP_EQ = 0, OP_X = 1, OP_I = 2, OP_D = 3 };
enum { ALG_NW = 0, ALG_SWG = 1, ALG_WFA = 2 };

static int32_t min2(int32_t a, int32_t b) { return a < b ? a : b; }

/* Run-length encode ops given in *reverse* order (last op first). */
static int32_t rle_reverse(const uint8_t *rev, int32_t nops, uint32_t *runs, int32_t cap) {
  int32_t nr = 0;
  int32_t t = nops - 1;
  while (t >= 0) {
    uint8_t op = rev[t];
    int32_t len = 0;
    while (t >= 0 && rev[t] == op) { ++len; --t; }
    if (nr >= cap) return -1;
    runs[nr++] = ((uint32_t)len << 4) | op;
  }
  return nr;
}

/* Linear-gap NW.  Returns 0 on success, -1 on allocation failure, -2 if the
 * traceback dead-ends (it cannot for valid penalties), -3 on CIGAR overflow. */
int oracle_nw(const uint8_t *P, int32_t m, const uint8_t *T, int32_t n, int32_t x, int32_t g,
              int32_t want_cigar, int32_t *score, uint32_t *runs, int32_t cap, int32_t *nruns) {
  int64_t W = (int64_t)n + 1;
  int32_t *H = (int32_t *)malloc(sizeof(int32_t) * (size_t)((int64_t)(m + 1) * W));
  if (!H) return -1;
#define AT(A, i, j) A[(int64_t)(i) * W + (j)]
  for (int32_t i = 0; i <= m; ++i) AT(H, i, 0) = i * g;
  for (int32_t j = 0; j <= n; ++j) AT(H, 0, j) = j * g;
  for (int32_t i = 1; i <= m; ++i)
    for (int32_t j = 1; j <= n; ++j) {
      int32_t c = P[i - 1] == T[j - 1] ? 0 : x;
      AT(H, i, j) = min2(AT(H, i - 1, j - 1) + c, min2(AT(H, i - 1, j) + g, AT(H, i, j - 1) + g));
    }
  *score = AT(H, m, n);
  *nruns = 0;
  int rc = 0;
  if (want_cigar) {
    uint8_t *rev = (uint8_t *)malloc((size_t)m + (size_t)n + 1);
    if (!rev) { free(H); return -1; }
    int32_t i = m, j = n, k = 0;
    while (i > 0 || j > 0) {
      int32_t h = AT(H, i, j);
      int mism = i > 0 && j > 0 && P[i - 1] != T[j - 1];
      if (mism && h == AT(H, i - 1, j - 1) + x) { rev[k++] = OP_X; --i; --j; }
      else if (i > 0 && h == AT(H, i - 1, j) + g) { rev[k++] = OP_I; --i; }
      else if (j > 0 && h == AT(H, i, j - 1) + g) { rev[k++] = OP_D; --j; }
      else if (i > 0 && j > 0 && !mism && h == AT(H, i - 1, j - 1)) { rev[k++] = OP_EQ; --i; --j; }
      else { rc = -2; break; }
    }
    if (rc == 0) {
      int32_t nr = rle_reverse(rev, k, runs, cap);
      if (nr < 0) rc = -3; else *nruns = nr;
    }
    free(rev);
  }
#undef AT
  free(H);
  return rc;
}

/* Affine-gap Gotoh (gap_open may be 0). Same return codes as oracle_nw. */
int oracle_gotoh(const uint8_t *P, int32_t m, const uint8_t *T, int32_t n, int32_t x, int32_t o,
                 int32_t e, int32_t want_cigar, int32_t *score, uint32_t *runs, int32_t cap,
                 int32_t *nruns) {
  int64_t W = (int64_t)n + 1;
  size_t cells = (size_t)((int64_t)(m + 1) * W);
  int32_t *H = (int32_t *)malloc(sizeof(int32_t) * cells);
  int32_t *E = (int32_t *)malloc(sizeof(int32_t) * cells);
  int32_t *F = (int32_t *)malloc(sizeof(int32_t) * cells);
  if (!H || !E || !F) { free(H); free(E); free(F); return -1; }
#define AT(A, i, j) A[(int64_t)(i) * W + (j)]
  AT(H, 0, 0) = 0; AT(E, 0, 0) = INF; AT(F, 0, 0) = INF;
  for (int32_t i = 1; i <= m; ++i) { AT(H, i, 0) = AT(E, i, 0) = o + i * e; AT(F, i, 0) = INF; }
  for (int32_t j = 1; j <= n; ++j) { AT(H, 0, j) = AT(F, 0, j) = o + j * e; AT(E, 0, j) = INF; }
  for (int32_t i = 1; i <= m; ++i)
    for (int32_t j = 1; j <= n; ++j) {
      int32_t c = P[i - 1] == T[j - 1] ? 0 : x;
      AT(E, i, j) = min2(AT(H, i - 1, j) + o + e, AT(E, i - 1, j) + e);
      AT(F, i, j) = min2(AT(H, i, j - 1) + o + e, AT(F, i, j - 1) + e);
      AT(H, i, j) = min2(AT(H, i - 1, j - 1) + c, min2(AT(E, i, j), AT(F, i, j)));
    }
  *score = AT(H, m, n);
  *nruns = 0;
  int rc = 0;
  if (want_cigar) {
    uint8_t *rev = (uint8_t *)malloc((size_t)m + (size_t)n + 1);
    if (!rev) { free(H); free(E); free(F); return -1; }
    int32_t i = m, j = n, k = 0;
    int state = 0; /* 0 H, 1 E, 2 F */
    while (i > 0 || j > 0) {
      if (state == 0) {
        int32_t h = AT(H, i, j);
        int mism = i > 0 && j > 0 && P[i - 1] != T[j - 1];
        if (mism && h == AT(H, i - 1, j - 1) + x) { rev[k++] = OP_X; --i; --j; }
        else if (i > 0 && h == AT(E, i, j)) state = 1;
        else if (j > 0 && h == AT(F, i, j)) state = 2;
        else if (i > 0 && j > 0 && !mism && h == AT(H, i - 1, j - 1)) { rev[k++] = OP_EQ; --i; --j; }
        else { rc = -2; break; }
      } else if (state == 1) {
        rev[k++] = OP_I;
        if (AT(E, i, j) == AT(H, i - 1, j) + o + e) state = 0;
        else if (i < 2 || AT(E, i, j) != AT(E, i - 1, j) + e) { rc = -2; break; }
        --i;
      } else {
        rev[k++] = OP_D;
        if (AT(F, i, j) == AT(H, i, j - 1) + o + e) state = 0;
        else if (j < 2 || AT(F, i, j) != AT(F, i, j - 1) + e) { rc = -2; break; }
        --j;
      }
    }
    if (rc == 0) {
      int32_t nr = rle_reverse(rev, k, runs, cap);
      if (nr < 0) rc = -3; else *nruns = nr;
    }
    free(rev);
  }
#undef AT
  free(H); free(E); free(F);
  return rc;
}

/* One pair under an algorithm and threshold.  status: 0 aligned, 1 rejected,
 * negative = oracle failure (see oracle_nw). */
int oracle_align_pair(const uint8_t *P, int32_t m, const uint8_t *T, int32_t n, int32_t alg,
                      int32_t x, int32_t o, int32_t e, int32_t max_score, int32_t want_cigar,
                      int32_t *score, int8_t *status, uint32_t *runs, int32_t cap, int32_t *nruns) {
  int32_t s = 0, nr = 0;
  int rc;
  if (alg == ALG_NW) rc = oracle_nw(P, m, T, n, x, e, want_cigar, &s, runs, cap, &nr);
  else rc = oracle_gotoh(P, m, T, n, x, o, e, want_cigar, &s, runs, cap, &nr);
  if (rc != 0) { *status = (int8_t)rc; *score = -1; *nruns = 0; return rc; }
  if (max_score >= 0 && s > max_score) { *status = 1; *score = -1; *nruns = 0; return 0; }
  *status = 0; *score = s; *nruns = nr;
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Batch driver: pairs are independent; a pthread pool takes chunks of     */
/* pairs dynamically.  Each pair's runs go to runs[slot_off[p] ...].       */
/* ---------------------------------------------------------------------- */
typedef struct {
  int64_t n;
  const uint8_t *pat; const int64_t *pat_off;
  const uint8_t *txt; const int64_t *txt_off;
  int32_t alg, x, o, e, max_score, want_cigar;
  int32_t *score; int8_t *status; uint32_t *runs; const int64_t *slot_off; int32_t *nruns;
  int64_t next; pthread_mutex_t mu;
} batch_job;

static void *batch_worker(void *arg) {
  batch_job *J = (batch_job *)arg;
  for (;;) {
    pthread_mutex_lock(&J->mu);
    int64_t a = J->next;
    J->next += 16;
    pthread_mutex_unlock(&J->mu);
    if (a >= J->n) break;
    int64_t b = a + 16 < J->n ? a + 16 : J->n;
    for (int64_t p = a; p < b; ++p) {
      int32_t m = (int32_t)(J->pat_off[p + 1] - J->pat_off[p]);
      int32_t n = (int32_t)(J->txt_off[p + 1] - J->txt_off[p]);
      int32_t cap = (int32_t)(J->slot_off[p + 1] - J->slot_off[p]);
      oracle_align_pair(J->pat + J->pat_off[p], m, J->txt + J->txt_off[p], n, J->alg, J->x, J->o,
                        J->e, J->max_score, J->want_cigar, &J->score[p], &J->status[p],
                        J->runs + J->slot_off[p], cap, &J->nruns[p]);
    }
  }
  return NULL;
}

int oracle_align_batch(int64_t n, const uint8_t *pat, const int64_t *pat_off, const uint8_t *txt,
                       const int64_t *txt_off, int32_t alg, int32_t x, int32_t o, int32_t e,
                       int32_t max_score, int32_t want_cigar, int32_t nthreads, int32_t *score,
                       int8_t *status, uint32_t *runs, const int64_t *slot_off, int32_t *nruns) {
  batch_job J = {n, pat, pat_off, txt, txt_off, alg, x, o, e, max_score, want_cigar,
                 score, status, runs, slot_off, nruns, 0, PTHREAD_MUTEX_INITIALIZER};
  if (nthreads < 1) nthreads = 1;
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
  if (!th) return -1;
  int started = 0;
  for (int t = 0; t < nthreads; ++t)
    if (pthread_create(&th[started], NULL, batch_worker, &J) == 0) ++started;
  if (started == 0) batch_worker(&J);
  for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
  free(th);
  return 0;
}
