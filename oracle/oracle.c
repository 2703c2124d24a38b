/*
 * oracle.c -- plain, slow, FP64 CPU reference of the PROJECTION hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant generator
 * with the GPU path.
 *
 * Paper: "PROJECTION Algorithm for Motif Finding on GPUs" (Clemente, Cabarle,
 * Adorna).  Each function cites the passage it follows.  Readings of passages
 * that are silent or garbled are listed beside the function that takes them.
 *
 * Layout conventions (plain, no packing):
 *   codes[]    one byte per symbol, all t sequences concatenated;
 *   off[t+1]   symbol offsets, sequence i is codes[off[i] .. off[i+1]);
 *   window     the l-mer of sequence i starting at a (0-based), a in
 *              [0, n_i - l]; windows are numbered w = 0..x-1 in (i, a) order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads of the OpenMP loops below (timing of the CPU baseline); returns the
 * number in use afterwards (1 without OpenMP). */
int or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ---------------------------------------------------------------------- */
/* Sec. 2 (notation) and Sec. 6 (integer equivalent of a k-mer): the DNA
 * letters map to A:0, C:1, T:2, G:3.  The paper only lists the first protein
 * letters (garbled); the reading taken is the conventional 20-letter order
 * A R N D C Q E G H I L K M F P S T W Y V.                                  */
static int code_of(int A, char ch)
{
    if (ch >= 'a' && ch <= 'z') ch = (char)(ch - 'a' + 'A');
    if (A == 4) {
        switch (ch) {
        case 'A': return 0;
        case 'C': return 1;
        case 'T': return 2;
        case 'G': return 3;
        default: return -1;
        }
    }
    if (A == 20) {
        const char *order = "ARNDCQEGHILKMFPSTWYV";
        for (int i = 0; i < 20; ++i)
            if (order[i] == ch) return i;
        return -1;
    }
    return -1;
}

char or_letter(int A, int code)
{
    if (A == 4) return "ACTG"[code];
    return "ARNDCQEGHILKMFPSTWYV"[code];
}

/* Returns -1 on success, else the index of the first symbol outside Sigma. */
int64_t or_encode(int A, const char *ascii, int64_t n, uint8_t *codes)
{
    for (int64_t g = 0; g < n; ++g) {
        int c = code_of(A, ascii[g]);
        if (c < 0) return g;
        codes[g] = (uint8_t)c;
    }
    return -1;
}

static int64_t windows_total(int t, const int64_t *off, int l)
{
    int64_t x = 0;
    for (int i = 0; i < t; ++i) x += (off[i + 1] - off[i]) - l + 1;
    return x;
}

int64_t or_num_windows(int t, const int64_t *off, int l) { return windows_total(t, off, l); }

/* ---------------------------------------------------------------------- */
/* Sec. 5, random projection h_k and Alg. 2 steps 2(b)-(c); Sec. 6, base-|Sigma|
 * integer of the projected k-mer, most significant symbol first (the example
 * "AAAAAAACG" -> 7 fixes the digit order).
 *
 * masks[j]: bit p set <=> window position p is projected in trial j.  The
 * projected positions are taken in ascending order (order preserved).
 * keys:   [m][x] or NULL;  counts: [m][A^k] or NULL.                       */
int or_hash(int A, int t, const int64_t *off, const uint8_t *codes, int l, int k,
            const uint32_t *masks, int m, uint32_t *keys, uint32_t *counts)
{
    /* a mask must keep exactly k of the l positions */
    for (int j = 0; j < m; ++j) {
        int pc = 0;
        for (int p = 0; p < 32; ++p)
            if (masks[j] >> p & 1u) pc += (p < l) ? 1 : 100;
        if (pc != k) return -1;
    }
    int64_t x = windows_total(t, off, l);
    uint64_t nb = 1;
    for (int q = 0; q < k; ++q) nb *= (uint64_t)A;
#pragma omp parallel for schedule(dynamic)
    for (int j = 0; j < m; ++j) {
        int pos[32];
        int kk = 0;
        for (int p = 0; p < l; ++p)
            if (masks[j] & (1u << p)) pos[kk++] = p;
        uint32_t *cnt = counts ? counts + (int64_t)j * (int64_t)nb : NULL;
        if (cnt) memset(cnt, 0, nb * sizeof(uint32_t));
        int64_t w = 0;
        for (int i = 0; i < t; ++i) {
            int64_t n_i = off[i + 1] - off[i];
            for (int64_t a = 0; a + l <= n_i; ++a, ++w) {
                uint64_t key = 0;
                for (int q = 0; q < kk; ++q)
                    key = key * (uint64_t)A + codes[off[i] + a + pos[q]];
                if (keys) keys[(int64_t)j * x + w] = (uint32_t)key;
                if (cnt) cnt[key] += 1;
            }
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Alg. 2 step 3, "identify enriched buckets": a bucket of trial j is enriched
 * when it holds at least s l-mers.  Readings: the l-mer itself counts (size
 * >= s); several l-mers of one sequence all count; one bucket per
 * (trial, key), listed in ascending (trial, key) order; members are window
 * numbers in ascending order.
 *
 * Output (truncated to the capacities, required totals in n_out[0..1]):
 *   bk[4*b + 0..3] = trial, key, size, first member slot.
 * Returns 0, or -3 when a capacity was too small.                          */
int or_select(int t, const int64_t *off, int l, int A, int k,
              const uint32_t *keys, const uint32_t *counts, int m, uint32_t s,
              uint32_t *bk, int64_t cap_b, uint32_t *members, int64_t cap_m,
              int64_t *n_out)
{
    int64_t x = windows_total(t, off, l);
    uint64_t nb = 1;
    for (int q = 0; q < k; ++q) nb *= (uint64_t)A;
    int64_t nbk = 0, nmem = 0;
    int64_t *slot = (int64_t *)malloc(nb * sizeof(int64_t));
    for (int j = 0; j < m; ++j) {
        const uint32_t *cnt = counts + (int64_t)j * (int64_t)nb;
        const uint32_t *kj = keys + (int64_t)j * x;
        for (uint64_t key = 0; key < nb; ++key) slot[key] = -1;
        for (uint64_t key = 0; key < nb; ++key) {
            if (cnt[key] >= s && cnt[key] > 0) {
                if (nbk < cap_b) {
                    bk[4 * nbk + 0] = (uint32_t)j;
                    bk[4 * nbk + 1] = (uint32_t)key;
                    bk[4 * nbk + 2] = cnt[key];
                    bk[4 * nbk + 3] = (uint32_t)nmem;
                }
                slot[key] = nmem;
                nbk += 1;
                nmem += cnt[key];
            }
        }
        /* stable placement: windows visited in ascending order */
        for (int64_t w = 0; w < x; ++w) {
            int64_t sl = slot[kj[w]];
            if (sl >= 0) {
                if (sl < cap_m) members[sl] = (uint32_t)w;
                slot[kj[w]] = sl + 1;
            }
        }
    }
    free(slot);
    n_out[0] = nbk;
    n_out[1] = nmem;
    return (nbk > cap_b || nmem > cap_m) ? -3 : 0;
}

/* The same enriched-bucket list without the |Sigma|^k count table (Alg. 2
 * step 3 for alphabets and k whose table does not fit; the paper's own answer
 * to that space problem is its K2 of Sec. 6).  Definition used here: sort
 * every trial's (key, window) pairs by key, then window; a run of equal keys
 * is one bucket, enriched when its length is at least s.  Same output order
 * and contents as or_select (buckets by (trial, key), members ascending).
 * Needs keys only.  Returns 0, -3 on a too small capacity, -2 on no memory. */
typedef struct { uint32_t key, w; } or_kw;

static int cmp_kw(const void *pa, const void *pb)
{
    const or_kw *a = (const or_kw *)pa, *b = (const or_kw *)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->w != b->w) return a->w < b->w ? -1 : 1;
    return 0;
}

int or_select_sorted(int t, const int64_t *off, int l, const uint32_t *keys, int m, uint32_t s,
                     uint32_t *bk, int64_t cap_b, uint32_t *members, int64_t cap_m, int64_t *n_out)
{
    int64_t x = windows_total(t, off, l);
    int64_t nbk = 0, nmem = 0;
    or_kw *v = (or_kw *)malloc((size_t)(x > 0 ? x : 1) * sizeof(or_kw));
    if (!v) return -2;
    for (int j = 0; j < m; ++j) {
        const uint32_t *kj = keys + (int64_t)j * x;
        for (int64_t w = 0; w < x; ++w) {
            v[w].key = kj[w];
            v[w].w = (uint32_t)w;
        }
        qsort(v, (size_t)x, sizeof(or_kw), cmp_kw);
        int64_t r0 = 0;
        while (r0 < x) {
            int64_t r1 = r0 + 1;
            while (r1 < x && v[r1].key == v[r0].key) ++r1;
            int64_t size = r1 - r0;
            if (size >= (int64_t)s) {
                if (nbk < cap_b) {
                    bk[4 * nbk + 0] = (uint32_t)j;
                    bk[4 * nbk + 1] = v[r0].key;
                    bk[4 * nbk + 2] = (uint32_t)size;
                    bk[4 * nbk + 3] = (uint32_t)nmem;
                }
                for (int64_t q = r0; q < r1; ++q)
                    if (nmem + (q - r0) < cap_m) members[nmem + (q - r0)] = v[q].w;
                nbk += 1;
                nmem += size;
            }
            r0 = r1;
        }
    }
    free(v);
    n_out[0] = nbk;
    n_out[1] = nmem;
    return (nbk > cap_b || nmem > cap_m) ? -3 : 0;
}

/* window number -> (sequence, start) */
static void window_site(int t, const int64_t *off, int l, int64_t w, int *i_out, int64_t *a_out)
{
    for (int i = 0; i < t; ++i) {
        int64_t L = (off[i + 1] - off[i]) - l + 1;
        if (w < L) { *i_out = i; *a_out = w; return; }
        w -= L;
    }
    *i_out = -1; *a_out = -1;
}

/* Sec. 2, profile matrix P(s): count of each letter in each column of the
 * alignment of the bucket's l-mers.  prof: [nb_use][A][l].                 */
void or_profile(int t, const int64_t *off, const uint8_t *codes, int l, int A,
                const uint32_t *bk, int64_t nbk, const uint32_t *members, uint32_t *prof)
{
    for (int64_t b = 0; b < nbk; ++b) {
        uint32_t *P = prof + b * A * l;
        memset(P, 0, sizeof(uint32_t) * A * l);
        for (uint32_t r = 0; r < bk[4 * b + 2]; ++r) {
            int i; int64_t a;
            window_site(t, off, l, members[bk[4 * b + 3] + r], &i, &a);
            for (int p = 0; p < l; ++p) P[codes[off[i] + a + p] * l + p] += 1;
        }
    }
}

/* Sec. 5.1 and Fig. 4: the initial model theta^0 is the column-letter
 * frequency of the bucket's alignment.  Reading (the paper prints zeros and
 * gives no pseudocounts): theta0 = (f + beta*bg) / (size + beta); beta = 0
 * gives the paper's raw frequencies.                                       */
void or_theta0(int A, int l, const uint32_t *prof, int64_t nbk, const double *bg,
               double beta, double *theta0)
{
    for (int64_t b = 0; b < nbk; ++b) {
        const uint32_t *P = prof + b * A * l;
        double size = 0;
        for (int c = 0; c < A; ++c) size += P[c * l + 0];
        for (int c = 0; c < A; ++c)
            for (int p = 0; p < l; ++p)
                theta0[b * A * l + c * l + p] = (P[c * l + p] + beta * bg[c]) / (size + beta);
    }
}

/* ---------------------------------------------------------------------- */
/* Sec. 5.1, EM refinement under the OOPS model (Sec. 2: one occurrence per
 * sequence).  The paper states neither step; the reading taken is the
 * standard OOPS EM of the works it cites (Lawrence & Reilly; Bailey), with a
 * uniform prior 1/L_i over the L_i = n_i - l + 1 starts and the background
 * fixed at bg:
 *
 *   W[c][p]  = ln theta[c][p] - ln bg[c]
 *   s_ia     = sum_p W[S_i[a+p]][p]                   (log-odds of start a)
 *   LSE_i    = ln sum_a exp(s_ia)
 *   Z_ia     = exp(s_ia - LSE_i)                      (E-step posterior)
 *   LLR      = sum_i (LSE_i - ln L_i)
 *   J        = LLR + beta * sum_{c,p} bg[c] ln theta[c][p]
 *   counts   c[c][p] = sum_{i,a} Z_ia [S_i[a+p] = c]   (M-step)
 *   theta'   = (counts + beta*bg) / (t + beta)
 *
 * J is the penalised likelihood that this EM never decreases (Dempster et
 * al.).  This function does one E-step for one model and exposes every
 * intermediate; s, Z: [x]; lse: [t].  Returns LLR.                          */
double or_estep(int t, const int64_t *off, const uint8_t *codes, int l, int A,
                const double *theta, const double *bg, double *s, double *Z, double *lse)
{
    double W[20 * 32];
    for (int c = 0; c < A; ++c)
        for (int p = 0; p < l; ++p) W[c * l + p] = log(theta[c * l + p]) - log(bg[c]);
    double llr = 0;
    int64_t w0 = 0;
    for (int i = 0; i < t; ++i) {
        int64_t L = (off[i + 1] - off[i]) - l + 1;
        double mx = -INFINITY;
        for (int64_t a = 0; a < L; ++a) {
            double v = 0;
            for (int p = 0; p < l; ++p) v += W[codes[off[i] + a + p] * l + p];
            s[w0 + a] = v;
            if (v > mx) mx = v;
        }
        double sum = 0;
        for (int64_t a = 0; a < L; ++a) sum += exp(s[w0 + a] - mx);
        double ls = mx + log(sum);
        if (lse) lse[i] = ls;
        for (int64_t a = 0; a < L; ++a) Z[w0 + a] = exp(s[w0 + a] - ls);
        llr += ls - log((double)L);
        w0 += L;
    }
    return llr;
}

/* The M-step above for one model given the posteriors Z: [x]. */
void or_mstep(int t, const int64_t *off, const uint8_t *codes, int l, int A,
              const double *Z, const double *bg, double beta, double *theta_new)
{
    double cnt[20 * 32];
    memset(cnt, 0, sizeof(cnt));
    int64_t w0 = 0;
    for (int i = 0; i < t; ++i) {
        int64_t L = (off[i + 1] - off[i]) - l + 1;
        for (int64_t a = 0; a < L; ++a)
            for (int p = 0; p < l; ++p) cnt[codes[off[i] + a + p] * l + p] += Z[w0 + a];
        w0 += L;
    }
    for (int c = 0; c < A; ++c)
        for (int p = 0; p < l; ++p)
            theta_new[c * l + p] = (cnt[c * l + p] + beta * bg[c]) / ((double)t + beta);
}

static double prior_term(int A, int l, const double *theta, const double *bg, double beta)
{
    if (beta == 0) return 0;
    double v = 0;
    for (int c = 0; c < A; ++c)
        for (int p = 0; p < l; ++p) v += bg[c] * log(theta[c * l + p]);
    return beta * v;
}

/* EM for B independent models, iters iterations, then a final E-step.
 *   theta0, theta_out: [B][A][l];  J, llr: [B][iters+1] (for theta^0..theta^iters);
 *   sites: [B][t], the start a maximising s_ia under theta^iters (first on ties). */
void or_em(int t, const int64_t *off, const uint8_t *codes, int l, int A,
           const double *theta0, const double *bg, int64_t B, int iters, double beta,
           double *theta_out, double *J, double *llr, int32_t *sites)
{
    int64_t x = windows_total(t, off, l);
#pragma omp parallel
    {
        double *s = (double *)malloc(sizeof(double) * (x > 0 ? x : 1));
        double *Z = (double *)malloc(sizeof(double) * (x > 0 ? x : 1));
        double th[20 * 32], th2[20 * 32];
#pragma omp for schedule(dynamic)
        for (int64_t b = 0; b < B; ++b) {
            memcpy(th, theta0 + b * A * l, sizeof(double) * A * l);
            for (int it = 0; it <= iters; ++it) {
                double v = or_estep(t, off, codes, l, A, th, bg, s, Z, NULL);
                llr[b * (iters + 1) + it] = v;
                J[b * (iters + 1) + it] = v + prior_term(A, l, th, bg, beta);
                if (it < iters) {
                    or_mstep(t, off, codes, l, A, Z, bg, beta, th2);
                    memcpy(th, th2, sizeof(double) * A * l);
                }
            }
            memcpy(theta_out + b * A * l, th, sizeof(double) * A * l);
            int64_t w0 = 0;
            for (int i = 0; i < t; ++i) {
                int64_t L = (off[i + 1] - off[i]) - l + 1;
                int64_t best = 0;
                for (int64_t a = 1; a < L; ++a)
                    if (s[w0 + a] > s[w0 + best]) best = a;
                sites[b * t + i] = (int32_t)best;
                w0 += L;
            }
        }
        free(s);
        free(Z);
    }
}

/* ---------------------------------------------------------------------- */
/* ZOOPS and TCM sequence models.  Sec. 2 names them beside OOPS: ZOOPS lets a
 * sequence hold at most one occurrence (possibly none), TCM any number.  The
 * paper gives no formulas; these are the two-component mixtures of the MEME
 * papers it cites, with the motif model theta, the fixed background bg, a
 * uniform start prior within a sequence and one mixing parameter `mix`:
 *
 * ZOOPS (mix = gamma, the prior probability that a sequence holds a site):
 *   P(S_i) / P_bg(S_i) = (1 - gamma) + (gamma / L_i) sum_a e^{s_ia}
 *   LLR_i = ln of that;  Z_ia = (gamma / L_i) e^{s_ia} / that ratio;
 *   q_i = sum_a Z_ia, the posterior probability that S_i holds a site.
 * TCM (mix = lambda, the probability that a window is an occurrence; windows
 * are treated as independent draws, overlaps included):
 *   per window  (1 - lambda) + lambda e^{s_ia};  LLR = sum over windows of its
 *   ln;  Z_ia = lambda e^{s_ia} / ((1 - lambda) + lambda e^{s_ia}).
 * M-step (both): counts c[c][p] = sum_{i,a} Z_ia [S_i[a+p] = c],
 *   theta' = (c + beta*bg) / (sum_{i,a} Z_ia + beta),
 *   ZOOPS gamma' = sum_{i,a} Z_ia / t;  TCM lambda' = sum_{i,a} Z_ia / x.
 * J = LLR + beta * sum bg ln theta, as for OOPS; the mixing parameter has no
 * prior (its update maximises the expected complete log-likelihood), so EM
 * still never decreases J.  ZOOPS with gamma = 1 is OOPS.
 * Sites: ZOOPS reports the best start of a sequence when q_i >= 1/2, else -1;
 * TCM the best start when that window's Z_ia >= 1/2, else -1 (one site per
 * sequence is reported even though TCM allows several).                     */
#define OR_OOPS 0
#define OR_ZOOPS 1
#define OR_TCM 2

/* ln(e^u + e^v), with e^{-inf} = 0 */
static double log_add(double u, double v)
{
    if (u == -INFINITY) return v;
    if (v == -INFINITY) return u;
    double m = u > v ? u : v;
    return m + log(exp(u - m) + exp(v - m));
}

/* One E-step of `model` for one model; s, Z: [x]; q: [t] (or NULL).
 * Returns LLR. */
double or_estep_model(int model, double mix, int t, const int64_t *off, const uint8_t *codes, int l, int A,
                      const double *theta, const double *bg, double *s, double *Z, double *q)
{
    if (model == OR_OOPS) {
        double llr = or_estep(t, off, codes, l, A, theta, bg, s, Z, NULL);
        if (q)
            for (int i = 0; i < t; ++i) q[i] = 1.0;
        return llr;
    }
    double W[20 * 32];
    for (int c = 0; c < A; ++c)
        for (int p = 0; p < l; ++p) W[c * l + p] = log(theta[c * l + p]) - log(bg[c]);
    const double lmix = log(mix), lnone = log(1.0 - mix);
    double llr = 0;
    int64_t w0 = 0;
    for (int i = 0; i < t; ++i) {
        int64_t L = (off[i + 1] - off[i]) - l + 1;
        for (int64_t a = 0; a < L; ++a) {
            double v = 0;
            for (int p = 0; p < l; ++p) v += W[codes[off[i] + a + p] * l + p];
            s[w0 + a] = v;
        }
        if (model == OR_ZOOPS) {
            double mx = -INFINITY;
            for (int64_t a = 0; a < L; ++a)
                if (s[w0 + a] > mx) mx = s[w0 + a];
            double sum = 0;
            for (int64_t a = 0; a < L; ++a) sum += exp(s[w0 + a] - mx);
            const double lsite = lmix - log((double)L) + mx + log(sum);
            const double li = log_add(lnone, lsite);
            for (int64_t a = 0; a < L; ++a) Z[w0 + a] = exp(lmix - log((double)L) + s[w0 + a] - li);
            if (q) q[i] = exp(lsite - li);
            llr += li;
        } else {
            for (int64_t a = 0; a < L; ++a) {
                const double li = log_add(lnone, lmix + s[w0 + a]);
                Z[w0 + a] = exp(lmix + s[w0 + a] - li);
                llr += li;
            }
            if (q) {
                double m = 0;
                for (int64_t a = 0; a < L; ++a) m += Z[w0 + a];
                q[i] = m;
            }
        }
        w0 += L;
    }
    return llr;
}

/* The M-step of `model` given the posteriors Z: theta_new, and *mix_new. */
void or_mstep_model(int model, int t, const int64_t *off, const uint8_t *codes, int l, int A, const double *Z,
                    const double *bg, double beta, double mix, double *theta_new, double *mix_new)
{
    double cnt[20 * 32];
    memset(cnt, 0, sizeof(cnt));
    double total = 0;
    int64_t w0 = 0;
    for (int i = 0; i < t; ++i) {
        int64_t L = (off[i + 1] - off[i]) - l + 1;
        for (int64_t a = 0; a < L; ++a) {
            for (int p = 0; p < l; ++p) cnt[codes[off[i] + a + p] * l + p] += Z[w0 + a];
            total += Z[w0 + a];
        }
        w0 += L;
    }
    if (model == OR_OOPS) total = (double)t;
    for (int c = 0; c < A; ++c)
        for (int p = 0; p < l; ++p) theta_new[c * l + p] = (cnt[c * l + p] + beta * bg[c]) / (total + beta);
    /* sum Z is at most t (ZOOPS) or x (TCM); rounding can pass that bound by
     * an ulp, which would make ln(1 - mix) undefined, so the update is capped
     * at 1 */
    if (model == OR_ZOOPS) *mix_new = fmin(1.0, total / (double)t);
    else if (model == OR_TCM) *mix_new = fmin(1.0, total / (double)w0);
    else *mix_new = mix;
}

/* EM of `model` for B independent models from theta0 and mix0; outputs as
 * or_em, plus mix_out[B] (the mixing parameter of the final E-step). */
void or_em_model(int model, double mix0, int t, const int64_t *off, const uint8_t *codes, int l, int A,
                 const double *theta0, const double *bg, int64_t B, int iters, double beta, double *theta_out,
                 double *mix_out, double *J, double *llr, int32_t *sites)
{
    int64_t x = windows_total(t, off, l);
#pragma omp parallel
    {
        double *s = (double *)malloc(sizeof(double) * (x > 0 ? x : 1));
        double *Z = (double *)malloc(sizeof(double) * (x > 0 ? x : 1));
        double *q = (double *)malloc(sizeof(double) * (t > 0 ? t : 1));
        double th[20 * 32], th2[20 * 32];
#pragma omp for schedule(dynamic)
        for (int64_t b = 0; b < B; ++b) {
            memcpy(th, theta0 + b * A * l, sizeof(double) * A * l);
            double mix = mix0;
            for (int it = 0; it <= iters; ++it) {
                double v = or_estep_model(model, mix, t, off, codes, l, A, th, bg, s, Z, q);
                llr[b * (iters + 1) + it] = v;
                J[b * (iters + 1) + it] = v + prior_term(A, l, th, bg, beta);
                if (it < iters) {
                    double mix2 = mix;
                    or_mstep_model(model, t, off, codes, l, A, Z, bg, beta, mix, th2, &mix2);
                    memcpy(th, th2, sizeof(double) * A * l);
                    mix = mix2;
                }
            }
            memcpy(theta_out + b * A * l, th, sizeof(double) * A * l);
            if (mix_out) mix_out[b] = mix;
            int64_t w0 = 0;
            for (int i = 0; i < t; ++i) {
                int64_t L = (off[i + 1] - off[i]) - l + 1;
                int64_t best = 0;
                for (int64_t a = 1; a < L; ++a)
                    if (s[w0 + a] > s[w0 + best]) best = a;
                int keep = 1;
                if (model == OR_ZOOPS) keep = q[i] >= 0.5;
                else if (model == OR_TCM) keep = Z[w0 + best] >= 0.5;
                sites[b * t + i] = keep ? (int32_t)best : -1;
                w0 += L;
            }
        }
        free(s);
        free(Z);
        free(q);
    }
}

/* ---------------------------------------------------------------------- */
/* Gibbs sampling as the local optimiser that refines a bucket instead of EM
 * (Sec. 1 and Sec. 3 name Gibbs sampling beside EM; the sampler is the site
 * sampler of Lawrence et al., cited by the paper).  The paper gives no
 * details; the reading used here:
 *   start  a_i = the best start of S_i under the bucket's theta0 (first on ties);
 *   sweep  for i = 0..t-1 in order: counts c of the other t-1 current sites,
 *          theta = (c + beta*bg) / (t - 1 + beta), weight of start a of S_i
 *          w_a = prod_p theta[S_i[a+p]][p] / bg[S_i[a+p]]; draw a_i with
 *          probability w_a / sum w, by the first a whose running sum of
 *          weights exceeds u * sum w (u uniform in [0,1));
 *   score  of an alignment, F = sum_{c,p} n_cp ln(theta_cp / bg_c) with n the
 *          counts of all t sites and theta = (n + beta*bg) / (t + beta);
 *   answer the alignment of largest F among the start and the end of every
 *          sweep (the earliest on ties), its theta and sites.
 * Random numbers: Philox4x64-10 (Salmon et al., SC'11), key {seed, 0},
 * counter {sweep, i, model, 0}; u = (first output word >> 11) * 2^-53.      */
static void philox_round(uint64_t c[4], const uint64_t k[2])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const unsigned __int128 p0 = (unsigned __int128)M0 * c[0];
    const unsigned __int128 p1 = (unsigned __int128)M1 * c[2];
    const uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    const uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    const uint64_t n0 = hi1 ^ c[1] ^ k[0], n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
}

void or_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint64_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        philox_round(c, k);
        k[0] += 0x9E3779B97F4A7C15ull;
        k[1] += 0xBB67AE8584CAA73Bull;
    }
    for (int q = 0; q < 4; ++q) out[q] = c[q];
}

double or_gibbs_uniform(uint64_t seed, int sweep, int i, int64_t model)
{
    const uint64_t ctr[4] = {(uint64_t)sweep, (uint64_t)i, (uint64_t)model, 0};
    const uint64_t key[2] = {seed, 0};
    uint64_t out[4];
    or_philox4x64(ctr, key, out);
    return (double)(out[0] >> 11) * (1.0 / 9007199254740992.0);
}

/* counts n[c][p] of the sites of every sequence except `skip` (-1: none) */
static void site_counts(int t, const int64_t *off, const uint8_t *codes, int l, const int32_t *site, int skip,
                        double *n)
{
    memset(n, 0, sizeof(double) * 20 * 32);
    for (int i = 0; i < t; ++i) {
        if (i == skip) continue;
        for (int p = 0; p < l; ++p) n[codes[off[i] + site[i] + p] * l + p] += 1.0;
    }
}

/* The weights of the starts of S_i given the other sites, scaled by the
 * largest (w[a] = e^{s_a - max_a s}); returns their sum. */
static double gibbs_raw_weights(int t, const int64_t *off, const uint8_t *codes, int l, int A, const double *bg,
                                double beta, const int32_t *site, int i, double *w)
{
    double n[20 * 32], W[20 * 32];
    site_counts(t, off, codes, l, site, i, n);
    for (int c = 0; c < A; ++c)
        for (int p = 0; p < l; ++p)
            W[c * l + p] = log((n[c * l + p] + beta * bg[c]) / ((double)(t - 1) + beta)) - log(bg[c]);
    const int64_t L = (off[i + 1] - off[i]) - l + 1;
    double mx = -INFINITY;
    for (int64_t a = 0; a < L; ++a) {
        double v = 0;
        for (int p = 0; p < l; ++p) v += W[codes[off[i] + a + p] * l + p];
        w[a] = v;
        if (v > mx) mx = v;
    }
    double sum = 0;
    for (int64_t a = 0; a < L; ++a) {
        w[a] = exp(w[a] - mx);
        sum += w[a];
    }
    return sum;
}

/* The sampler's conditional distribution for sequence i: w[a] / sum w. */
void or_gibbs_weights(int t, const int64_t *off, const uint8_t *codes, int l, int A, const double *bg, double beta,
                      const int32_t *site, int i, double *w)
{
    const double sum = gibbs_raw_weights(t, off, codes, l, A, bg, beta, site, i, w);
    const int64_t L = (off[i + 1] - off[i]) - l + 1;
    for (int64_t a = 0; a < L; ++a) w[a] /= sum;
}

/* F of the alignment `site` and its theta */
double or_alignment_score(int t, const int64_t *off, const uint8_t *codes, int l, int A, const double *bg,
                          double beta, const int32_t *site, double *theta)
{
    double n[20 * 32];
    site_counts(t, off, codes, l, site, -1, n);
    double F = 0;
    for (int c = 0; c < A; ++c)
        for (int p = 0; p < l; ++p) {
            const double th = (n[c * l + p] + beta * bg[c]) / ((double)t + beta);
            if (theta) theta[c * l + p] = th;
            if (n[c * l + p] > 0) F += n[c * l + p] * log(th / bg[c]);
        }
    return F;
}

/* Gibbs refinement of B models: theta_out [B][A][l], F [B][sweeps+1] (F of
 * the start and after each sweep), sites [B][t] of the best alignment.
 * Returns 0, or -1 when beta <= 0. */
int or_gibbs(int t, const int64_t *off, const uint8_t *codes, int l, int A, const double *theta0, const double *bg,
             int64_t B, int sweeps, double beta, uint64_t seed, double *theta_out, double *F, int32_t *sites)
{
    if (!(beta > 0)) return -1;
    int64_t x = windows_total(t, off, l);
    int64_t Lmax = 1;
    for (int i = 0; i < t; ++i)
        if ((off[i + 1] - off[i]) - l + 1 > Lmax) Lmax = (off[i + 1] - off[i]) - l + 1;
#pragma omp parallel
    {
        double *s = (double *)malloc(sizeof(double) * (x > 0 ? x : 1));
        double *Z = (double *)malloc(sizeof(double) * (x > 0 ? x : 1));
        double *w = (double *)malloc(sizeof(double) * Lmax);
        int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * t);
        int32_t *bst = (int32_t *)malloc(sizeof(int32_t) * t);
#pragma omp for schedule(dynamic)
        for (int64_t b = 0; b < B; ++b) {
            /* start: the best start of every sequence under theta0 */
            or_estep(t, off, codes, l, A, theta0 + b * A * l, bg, s, Z, NULL);
            int64_t w0 = 0;
            for (int i = 0; i < t; ++i) {
                int64_t L = (off[i + 1] - off[i]) - l + 1, best = 0;
                for (int64_t a = 1; a < L; ++a)
                    if (s[w0 + a] > s[w0 + best]) best = a;
                cur[i] = (int32_t)best;
                w0 += L;
            }
            double Fb = or_alignment_score(t, off, codes, l, A, bg, beta, cur, NULL);
            F[b * (sweeps + 1)] = Fb;
            memcpy(bst, cur, sizeof(int32_t) * t);
            for (int r = 0; r < sweeps; ++r) {
                for (int i = 0; i < t; ++i) {
                    const int64_t L = (off[i + 1] - off[i]) - l + 1;
                    const double tot = gibbs_raw_weights(t, off, codes, l, A, bg, beta, cur, i, w);
                    const double target = or_gibbs_uniform(seed, r, i, b) * tot;
                    int64_t pick = L - 1;
                    double run = 0;
                    for (int64_t a = 0; a < L; ++a) {
                        run += w[a];
                        if (run > target) {
                            pick = a;
                            break;
                        }
                    }
                    cur[i] = (int32_t)pick;
                }
                const double Fr = or_alignment_score(t, off, codes, l, A, bg, beta, cur, NULL);
                F[b * (sweeps + 1) + r + 1] = Fr;
                if (Fr > Fb) {
                    Fb = Fr;
                    memcpy(bst, cur, sizeof(int32_t) * t);
                }
            }
            or_alignment_score(t, off, codes, l, A, bg, beta, bst, theta_out + b * A * l);
            memcpy(sites + b * t, bst, sizeof(int32_t) * t);
        }
        free(s);
        free(Z);
        free(w);
        free(cur);
        free(bst);
    }
    return 0;
}

/* Sec. 5.1: the model with the highest objective is the answer.  Readings:
 * the objective is J(theta^iters); ties go to the lowest bucket index (the
 * lowest (trial, key)); the consensus takes in each column the letter of
 * largest probability, the lowest code on ties (Sec. 2 lets ties be broken
 * arbitrarily).  NaN objectives never win.  Returns the bucket index or -1. */
int64_t or_best(const double *J, int64_t B, int iters, const double *theta, int A, int l,
                char *consensus)
{
    int64_t best = -1;
    for (int64_t b = 0; b < B; ++b) {
        double v = J[b * (iters + 1) + iters];
        if (v != v) continue;
        if (best < 0 || v > J[best * (iters + 1) + iters]) best = b;
    }
    if (best >= 0 && consensus) {
        const double *th = theta + best * A * l;
        for (int p = 0; p < l; ++p) {
            int bc = 0;
            for (int c = 1; c < A; ++c)
                if (th[c * l + p] > th[bc * l + p]) bc = c;
            consensus[p] = or_letter(A, bc);
        }
        consensus[l] = 0;
    }
    return best;
}

/* ---------------------------------------------------------------------- */
/* Projection tables from a seed (Sec. 6: l-k positions *not* to project are
 * drawn on the host).  Generator: the minimal standard generator of Park and
 * Miller (the paper's cited RNG), x <- 16807 x mod (2^31 - 1).  Reading of
 * "l-k random numbers in range [0,l]": l-k distinct positions from
 * {0..l-1}, drawn by a partial Fisher-Yates shuffle of the identity
 * permutation with index i + (r mod (l - i)).  The state for trial j starts
 * at 1 + (seed + j) mod (2^31 - 2), so every trial has its own stream.     */
static uint32_t pm_next(uint64_t *state)
{
    *state = (*state * 16807u) % 2147483647u;
    return (uint32_t)*state;
}

uint32_t or_parkmiller(uint64_t seed, int n)
{
    uint64_t st = seed;
    uint32_t v = 0;
    for (int i = 0; i < n; ++i) v = pm_next(&st);
    return v;
}

void or_masks(uint64_t seed, int l, int k, int m, uint32_t *masks)
{
    for (int j = 0; j < m; ++j) {
        uint64_t st = 1 + (seed + (uint64_t)j) % 2147483646u;
        int perm[32];
        for (int p = 0; p < l; ++p) perm[p] = p;
        uint32_t mask = (l == 32) ? 0xffffffffu : ((1u << l) - 1u);
        for (int i = 0; i < l - k; ++i) {
            int r = i + (int)(pm_next(&st) % (uint32_t)(l - i));
            int tmp = perm[i]; perm[i] = perm[r]; perm[r] = tmp;
            mask &= ~(1u << perm[i]);
        }
        masks[j] = mask;
    }
}
