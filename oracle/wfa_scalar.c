/*
 * Scalar CPU wavefront algorithm (WFA), gap-affine.  TEST INFRASTRUCTURE
 * ONLY: it pins the Gotoh oracle (same optimum, same canonical CIGAR) and
 * counts the wavefront work a pair needs.  It shares no code with the Gotoh
 * oracle nor with the GPU library.
 *
 * Paper: System and Methods, "Wavefront Algorithm (WFA)": successive
 * furthest-reaching wavefronts, one per score s, until the alignment reaches
 * the end cell; O(n s) work.  The recurrences below are the affine-gap
 * wavefront recurrences restated on offsets j (text position) along
 * diagonals k = j - i:
 *   I_s[k] = max(M_{s-o-e}[k+1], I_{s-e}[k+1])          (consumes P)
 *   D_s[k] = max(M_{s-o-e}[k-1], D_{s-e}[k-1]) + 1      (consumes T)
 *   M_s[k] = max(M_{s-x}[k] + 1, I_s[k], D_s[k])
 * then every valid M_s[k] is extended along matching bases.  A candidate is
 * invalid when it leaves the table (j > n or i = j - k > m).  M_0[0] =
 * extend(0).  The first s with M_s[n-m] >= n is the optimum.  With
 * max_score >= 0 the search stops (REJECTED) once s exceeds it.
 *
 * WFA-adaptive (paper: same subsection -- a heuristic variant that drops
 * outer diagonals unlikely to lead to the optimum; its rule is not spelled
 * out there, so the reading below is this library's, with the cited WFA
 * work's usual parameters as defaults): after score s is computed and
 * extended (and has not reached the end cell), if its range holds at least
 * min_len diagonals, each diagonal k with an M offset f gets the distance
 * d(k) = max(m - (f - k), n - f) -- the bases still to align along the longer
 * side -- and diagonals are removed from each end of the range, inwards, as
 * long as their M is absent or d(k) - min_k d(k) > max_dist.  The removed
 * cells of M, I and D no longer exist for later scores (nor for the
 * backtrace).  The result is a valid alignment whose cost is at least the
 * optimum.  min_len <= 0 turns the reduction off (exact WFA).
 *
 * Backtrace (reproduces the Gotoh oracle's canonical CIGAR): from M at
 * (s,k,f) let f0 = max of the three candidates; emit f - f0 '=' ops, then the
 * op of the first candidate attaining f0 in the order X, I, D.  From I (or D)
 * prefer the open source M_{s-o-e} over the extend source when both attain the
 * value.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NEG (INT32_MIN / 4)
enum { OP_EQ = 0, OP_X = 1, OP_I = 2, OP_D = 3 };

typedef struct {
  int32_t lo, hi; /* diagonal range; empty wavefront when lo > hi */
  int32_t base;   /* diagonal of the arrays' first entry (lo before any reduction) */
  int32_t *M, *I, *D; /* NULL when the component is null */
} wavefront;

static int32_t wf_get(const wavefront *w, const int32_t *a, int32_t k) {
  if (!a || k < w->lo || k > w->hi) return NEG;
  return a[k - w->base];
}

static int32_t max2(int32_t a, int32_t b) { return a > b ? a : b; }

/* Work of the last call, the units in which the wavefront algorithm's cost
 * is stated (O(n s): one unit per diagonal of every wavefront it computes).
 *   cells:      the widths hi_s - lo_s + 1 of every non-null wavefront,
 *               s = 0 (one diagonal) included;
 *   wavefronts: the non-null wavefronts;
 *   compared:   bases compared by the extensions, one per matching base plus
 *               one for the mismatch that stops a run (none when a run stops
 *               at the end of either sequence);
 *   words:      the same comparisons taken 32 bases at a time: a run of r
 *               matches costs floor(r / 32) + 1 words when a mismatch stops
 *               it and ceil(r / 32) when it stops at an end;
 *   lo_min, hi_max: the outermost diagonals any wavefront spans;
 *   dropped:    (adaptive) diagonals removed by the reduction. */
typedef struct { int64_t cells, compared, wavefronts, words; int32_t lo_min, hi_max; int64_t dropped; } wfa_stats;

static int wfa_run(const uint8_t *P, int32_t m, const uint8_t *T, int32_t n, int32_t x, int32_t o,
                   int32_t e, int32_t max_score, int32_t want_cigar, int32_t min_len, int32_t max_dist,
                   int32_t *score, int8_t *status, uint32_t *runs, int32_t cap, int32_t *nruns,
                   wfa_stats *st) {
  int32_t oe = o + e;
  int32_t cap_s = 64;
  wavefront *W = (wavefront *)calloc((size_t)cap_s, sizeof(wavefront));
  if (!W) return -1;
  wfa_stats S = {0, 0, 0, 0, 0, 0, 0};
  int32_t kend = n - m;
  int32_t s = 0;
  int rc = 0, done = 0;
  *nruns = 0;
  /* no alignment costs more than (m + n) ops at max(x, o + e) each: an
   * adaptive search that passes that has lost the end cell (it cannot, with
   * the rule above; the bound keeps a broken variant from running on) */
  const int64_t s_hard = (int64_t)(m + n) * max2(x, oe) + 1;
  for (;; ++s) {
    if (max_score >= 0 && s > max_score) break;
    if (min_len > 0 && s > s_hard) { rc = -4; break; }
    if (s >= cap_s) {
      int32_t nc = cap_s * 2;
      wavefront *nw = (wavefront *)realloc(W, sizeof(wavefront) * (size_t)nc);
      if (!nw) { rc = -1; break; }
      memset(nw + cap_s, 0, sizeof(wavefront) * (size_t)(nc - cap_s));
      W = nw; cap_s = nc;
    }
    wavefront *w = &W[s];
    w->lo = 1; w->hi = 0;
    const wavefront *wx = s - x >= 0 ? &W[s - x] : NULL;
    const wavefront *wo = s - oe >= 0 ? &W[s - oe] : NULL;
    const wavefront *we = s - e >= 0 ? &W[s - e] : NULL;
    if (s == 0) {
      w->lo = w->hi = w->base = 0;
      w->M = (int32_t *)malloc(sizeof(int32_t));
      if (!w->M) { rc = -1; break; }
      w->M[0] = 0;
      S.cells += 1;
    } else {
      int has_x = wx && wx->M, has_o = wo && wo->M, has_ie = we && we->I, has_de = we && we->D;
      if (!has_x && !has_o && !has_ie && !has_de) continue;
      int32_t lo = INT32_MAX, hi = INT32_MIN;
      if (has_x) { lo = lo < wx->lo ? lo : wx->lo; hi = hi > wx->hi ? hi : wx->hi; }
      if (has_o) { lo = lo < wo->lo ? lo : wo->lo; hi = hi > wo->hi ? hi : wo->hi; }
      if (has_ie || has_de) { lo = lo < we->lo ? lo : we->lo; hi = hi > we->hi ? hi : we->hi; }
      lo -= 1; hi += 1;
      if (lo < -m) lo = -m;
      if (hi > n) hi = n;
      if (lo > hi) continue;
      int32_t width = hi - lo + 1;
      w->lo = lo; w->hi = hi; w->base = lo;
      w->M = (int32_t *)malloc(sizeof(int32_t) * (size_t)width);
      w->I = (int32_t *)malloc(sizeof(int32_t) * (size_t)width);
      w->D = (int32_t *)malloc(sizeof(int32_t) * (size_t)width);
      if (!w->M || !w->I || !w->D) { rc = -1; break; }
      for (int32_t k = lo; k <= hi; ++k) {
        int32_t vi = max2(has_o ? wf_get(wo, wo->M, k + 1) : NEG, has_ie ? wf_get(we, we->I, k + 1) : NEG);
        if (vi >= 0 && vi - k > m) vi = NEG;
        int32_t vd = max2(has_o ? wf_get(wo, wo->M, k - 1) : NEG, has_de ? wf_get(we, we->D, k - 1) : NEG);
        if (vd >= 0) { vd += 1; if (vd > n) vd = NEG; } else vd = NEG;
        int32_t vx = has_x ? wf_get(wx, wx->M, k) : NEG;
        if (vx >= 0) { vx += 1; if (vx > n || vx - k > m) vx = NEG; } else vx = NEG;
        if (vi < 0) vi = NEG;
        w->I[k - lo] = vi;
        w->D[k - lo] = vd;
        w->M[k - lo] = max2(vx, max2(vi, vd));
      }
      S.cells += width;
    }
    S.wavefronts += 1;
    if (w->lo < S.lo_min) S.lo_min = w->lo;
    if (w->hi > S.hi_max) S.hi_max = w->hi;
    /* extend */
    for (int32_t k = w->lo; k <= w->hi; ++k) {
      int32_t f = w->M[k - w->base];
      if (f < 0) continue;
      int32_t i = f - k, j = f, run = 0;
      while (i < m && j < n && P[i] == T[j]) { ++i; ++j; ++run; }
      S.compared += run;
      if (i < m && j < n) {
        S.compared += 1;
        S.words += run / 32 + 1;
      } else {
        S.words += (run + 31) / 32;
      }
      w->M[k - w->base] = j;
    }
    if (kend >= w->lo && kend <= w->hi && w->M[kend - w->base] >= n) { done = 1; break; }
    if (min_len > 0 && w->hi - w->lo + 1 >= min_len) {
      /* adaptive reduction (see the header) */
      int32_t dmin = INT32_MAX;
      for (int32_t k = w->lo; k <= w->hi; ++k) {
        int32_t f = w->M[k - w->base];
        if (f < 0) continue;
        int32_t d = max2(m - (f - k), n - f);
        if (d < dmin) dmin = d;
      }
      if (dmin != INT32_MAX) {
        /* (the diagonal of distance dmin always stays; the bounds only
         * guard the loops) */
        int32_t lo = w->lo, hi = w->hi;
        while (lo < hi) {
          int32_t f = w->M[lo - w->base];
          if (f >= 0 && max2(m - (f - lo), n - f) - dmin <= max_dist) break;
          ++lo;
        }
        while (hi > lo) {
          int32_t f = w->M[hi - w->base];
          if (f >= 0 && max2(m - (f - hi), n - f) - dmin <= max_dist) break;
          --hi;
        }
        S.dropped += (int64_t)(lo - w->lo) + (int64_t)(w->hi - hi);
        w->lo = lo;
        w->hi = hi;
      }
    }
  }
  if (rc == 0 && !done) {
    *score = -1; *status = 1;
  } else if (rc == 0) {
    *score = s; *status = 0;
    if (want_cigar) {
      uint8_t *rev = (uint8_t *)malloc((size_t)m + (size_t)n + 1);
      if (!rev) rc = -1;
      int32_t nops = 0, cs = s, k = kend, comp = 0; /* comp: 0 M, 1 I, 2 D */
      int32_t f = n;
      while (rc == 0) {
        if (comp == 0) {
          if (cs == 0) { /* start wavefront: only matches from (0,0) */
            for (int32_t t = 0; t < f; ++t) rev[nops++] = OP_EQ;
            break;
          }
          const wavefront *w = &W[cs];
          const wavefront *wx = cs - x >= 0 ? &W[cs - x] : NULL;
          int32_t vx = wx && wx->M ? wf_get(wx, wx->M, k) : NEG;
          if (vx >= 0) { vx += 1; if (vx > n || vx - k > m) vx = NEG; } else vx = NEG;
          int32_t vi = wf_get(w, w->I, k), vd = wf_get(w, w->D, k);
          int32_t f0 = max2(vx, max2(vi, vd));
          if (f0 < 0) { rc = -2; break; }
          for (int32_t t = f0; t < f; ++t) rev[nops++] = OP_EQ;
          if (vx == f0) { rev[nops++] = OP_X; cs -= x; f = f0 - 1; }
          else if (vi == f0) { comp = 1; f = f0; }
          else { comp = 2; f = f0; }
        } else if (comp == 1) {
          rev[nops++] = OP_I;
          const wavefront *wo = cs - oe >= 0 ? &W[cs - oe] : NULL;
          int32_t vo = wo && wo->M ? wf_get(wo, wo->M, k + 1) : NEG;
          if (vo == f) { comp = 0; cs -= oe; }
          else { cs -= e; }
          k += 1;
        } else {
          rev[nops++] = OP_D;
          const wavefront *wo = cs - oe >= 0 ? &W[cs - oe] : NULL;
          int32_t vo = wo && wo->M ? wf_get(wo, wo->M, k - 1) : NEG;
          if (vo >= 0 && vo + 1 == f) { comp = 0; cs -= oe; }
          else { cs -= e; }
          k -= 1; f -= 1;
        }
        if (cs < 0) { rc = -2; break; }
      }
      if (rc == 0) {
        /* run-length encode the reversed op list */
        int32_t nr = 0, t = nops - 1;
        while (t >= 0) {
          uint8_t op = rev[t];
          int32_t len = 0;
          while (t >= 0 && rev[t] == op) { ++len; --t; }
          if (nr >= cap) { rc = -3; break; }
          runs[nr++] = ((uint32_t)len << 4) | op;
        }
        if (rc == 0) *nruns = nr;
      }
      free(rev);
    }
  }
  for (int32_t t = 0; t < cap_s; ++t) { free(W[t].M); free(W[t].I); free(W[t].D); }
  free(W);
  if (st) *st = S;
  if (rc != 0) { *score = -1; *status = (int8_t)rc; }
  return rc;
}

int oracle_wfa(const uint8_t *P, int32_t m, const uint8_t *T, int32_t n, int32_t x, int32_t o,
               int32_t e, int32_t max_score, int32_t want_cigar, int32_t *score, int8_t *status,
               uint32_t *runs, int32_t cap, int32_t *nruns, wfa_stats *st) {
  return wfa_run(P, m, T, n, x, o, e, max_score, want_cigar, 0, 0, score, status, runs, cap, nruns, st);
}

int oracle_wfa_adaptive(const uint8_t *P, int32_t m, const uint8_t *T, int32_t n, int32_t x, int32_t o,
                        int32_t e, int32_t max_score, int32_t want_cigar, int32_t min_len, int32_t max_dist,
                        int32_t *score, int8_t *status, uint32_t *runs, int32_t cap, int32_t *nruns,
                        wfa_stats *st) {
  return wfa_run(P, m, T, n, x, o, e, max_score, want_cigar, min_len, max_dist, score, status, runs, cap,
                 nruns, st);
}
