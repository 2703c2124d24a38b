/*
 * projmotif.h -- C ABI of the MI355X (gfx950) PROJECTION motif-finding path.
 *
 * Paper: "PROJECTION Algorithm for Motif Finding on GPUs" (Clemente, Cabarle,
 * Adorna).  The problem statement (Sec. 2; Alg. 2 and Alg. 3 INPUT/OUTPUT)
 * fixes the arguments: sequences S_1..S_t over an alphabet Sigma, motif
 * length l, projection size k, bucket threshold s, number of trials m.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function returns an int status: PM_OK (0) or a negative PM_E*
 *    code; pm_last_error() then gives a message (thread-local).  No C++
 *    exception crosses this boundary.
 *  - Pointers documented "device" are HIP device addresses; "host" are host
 *    addresses.  The caller owns every buffer: the library never frees caller
 *    memory, and the device-pointer entry points allocate nothing.
 *  - Device-pointer entry points are asynchronous on `stream` (a hipStream_t
 *    passed as void*, NULL = the null stream).  Host-side argument checks
 *    return an error before anything is enqueued.  Conditions that only the
 *    device can see (a symbol outside Sigma, a bad projection mask, a capacity
 *    that is too small) are OR-ed into a caller-provided device word `status`
 *    (PM_STATUS_* bits; may be NULL) and the affected outputs are left
 *    unwritten or truncated as documented.
 *  - Counts that depend on the data (number of enriched buckets) are written
 *    to device memory; later calls read them from there (`n_dev`), so a whole
 *    pass needs no host synchronisation.
 *  - Symbol codes: DNA A:0 C:1 T:2 G:3 (Sec. 6); protein in the order
 *    A R N D C Q E G H I L K M F P S T W Y V (the paper lists the protein
 *    alphabet only in part).  Lower-case letters are accepted.
 *  - Window (l-mer) numbering: window w is the l-mer of sequence i starting
 *    at a (0-based), numbered in (i, a) order; x = sum_i (n_i - l + 1).
 *    Sites are 0-based (the paper's a_i are 1-based, Sec. 2).
 */
#ifndef PROJMOTIF_H
#define PROJMOTIF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PM_OK 0
#define PM_EINVAL (-1)     /* invalid argument (l, k, s, m, alphabet, sizes) */
#define PM_ERANGE (-2)     /* supported but too large: |Sigma|^k, LDS budget */
#define PM_ECAPACITY (-3)  /* an output capacity was too small */
#define PM_EDEVICE (-4)    /* a HIP runtime error */

#define PM_STATUS_BAD_SYMBOL 1u  /* pm_pack met a byte outside Sigma */
#define PM_STATUS_BAD_MASK 2u    /* a projection mask does not keep exactly k of l positions */
#define PM_STATUS_CAPACITY 4u    /* bucket_select outputs truncated */

#define PM_DNA 4
#define PM_PROTEIN 20

/* EM arithmetic (em_refine `precision`).  In every form the per-sequence
 * log-sum-exp is FP64: each window's term exp(s_ia - ref) is formed in the
 * form's precision and accumulated over the sequence in FP64 (the DNA
 * matrix-core forms first add the eight terms a lane holds for one 32-window
 * pair in FP32, at most 3 * 2^-24 relative error), lane partials are
 * combined in FP64, the logarithm is FP64, and LLR, J and the final
 * comparison of models are FP64. */
#define PM_FP64 0  /* every step in FP64 */
#define PM_FP32 1  /* scores, exponentials, posteriors and counts in FP32 */
#define PM_F16X2 2 /* DNA only: E- and M-step on FP16 matrix cores with every non-0/1
                      operand split into two FP16 halves (about 22 significant bits,
                      exact products, FP32 sums) */
#define PM_F16 3   /* the precision form, DNA and protein (l <= 24, t <= 64,
                      n_i <= 2048 for protein): the same contractions with one FP16
                      value per operand (11 significant bits) and FP32 accumulation;
                      results carry FP16-level error against FP64, which the caller
                      measures and states */

/* Encoded sequences.  Host fields describe the device arrays. */
typedef struct pm_seqs {
    int32_t alphabet;        /* |Sigma|: PM_DNA or PM_PROTEIN */
    int32_t t;               /* number of sequences, >= 1 */
    int64_t n_total;         /* host: sum of the lengths n_i */
    int32_t n_min;           /* host: shortest n_i */
    int32_t n_max;           /* host: longest n_i */
    const int64_t *offsets;  /* device [t+1]: offsets[0] = 0, sequence i is symbols
                                offsets[i] .. offsets[i+1]-1 of the concatenation */
    const uint32_t *packed;  /* device [pm_packed_words(alphabet, n_total)] from pm_pack */
} pm_seqs;

/* One enriched bucket (Alg. 2 step 3). */
typedef struct pm_bucket {
    uint32_t trial; /* trial j in [0, m) */
    uint32_t key;   /* base-|Sigma| integer of the projected k-mer (Sec. 6) */
    uint32_t size;  /* number of l-mers hashed to it (>= s) */
    uint32_t first; /* index of its first member in the members array */
} pm_bucket;

const char *pm_version(void);
const char *pm_last_error(void);

/* Number of uint32 words pm_pack writes for n_total symbols: 16 DNA or 6
 * protein symbols per word, first symbol in the most significant bits, plus
 * four zero words of padding at the end. */
int64_t pm_packed_words(int32_t alphabet, int64_t n_total);

/* a1 -- encode and pack (Sec. 6: the one-to-one map of letters to integers;
 * Sec. 6: sequences passed to the device as flat arrays).
 *   ascii   device [n_total] bytes, the t sequences concatenated
 *   packed  device [pm_packed_words(alphabet, n_total)], fully written
 * A byte outside Sigma is encoded as code 0 and sets PM_STATUS_BAD_SYMBOL. */
int pm_pack(int32_t alphabet, const uint8_t *ascii, int64_t n_total, uint32_t *packed,
            uint32_t *status, void *stream);

/* a2 -- projection tables on the host (Sec. 6: the l-k positions not to
 * project are drawn on the host).  Park-Miller minimal standard generator
 * (the paper's cited RNG); trial j uses the stream started at
 * 1 + (seed + j) mod (2^31 - 2) and a partial Fisher-Yates shuffle.
 *   masks  host [m]; bit p set <=> window position p is projected. */
int pm_masks_from_seed(uint64_t seed, int32_t l, int32_t k, int32_t m, uint32_t *masks);

/* Sec. 5, choice of the parameters when not given: k = l - d - 1;
 * s = max(3, ceil(2 x / |Sigma|^k)) (twice the mean bucket size, the paper
 * falling back to 3-4 when that mean is tiny); m = ceil(log(1-q) / log B(s)),
 * B(s) = P[Binomial(t, p_hat) < s], p_hat = C(l-d,k) / C(l,k).  Host only. */
int pm_auto_params(int32_t alphabet, int32_t t, int64_t x, int32_t l, int32_t d, double q,
                   int32_t *k, int32_t *s, int32_t *m);

/* a3 + a4 -- Alg. 2 steps 2(b) and 2(c): project every l-mer onto the
 * positions kept by each trial's mask (Sec. 5, order preserved) and hash the
 * k-mer to its base-|Sigma| integer, most significant symbol first (Sec. 6,
 * "AAAAAAACG" -> 7); count the l-mers of every bucket (PROJECTION1, Sec. 5.2).
 *   masks   device [m] (popcount k, below 2^l; otherwise PM_STATUS_BAD_MASK
 *           and that trial's outputs are not written)
 *   keys    device [m][x] uint32, or NULL
 *   counts  device [m][|Sigma|^k] uint32, or NULL (at least one non-NULL)
 * Limits: 1 <= k <= l <= 32, l <= n_min, |Sigma|^k <= 2^24 when counts are
 * requested (< 2^32 for keys only). */
int projection_hash(const pm_seqs *S, int32_t l, int32_t k, const uint32_t *masks, int32_t m,
                    uint32_t *keys, uint32_t *counts, uint32_t *status, void *stream);

/* Workspace bytes bucket_select needs for m trials of |Sigma|^k bins (a
 * per-trial bitmap of passing keys and per-trial totals; the member cursors
 * live in LDS, so cap_buckets does not change the size); 0 when the alphabet
 * is not 4 or 20 or |Sigma|^k exceeds 2^19. */
size_t pm_select_workspace(int32_t alphabet, int32_t k, int32_t m, int64_t cap_buckets);

/* a5 -- Alg. 2 step 3 and Sec. 6 (a bucket passes when it holds at least s
 * l-mers): list every (trial, key) with counts >= s, ascending by (trial,
 * key), and the member windows of each, ascending.
 *   keys, counts  device, as written by projection_hash
 *   buckets       device [cap_buckets]
 *   members       device [cap_members] window numbers
 *   n_out         device int64[2]: required number of buckets and members
 *                 (may exceed the capacities: then the lists are truncated to
 *                 their first entries and PM_STATUS_CAPACITY is set)
 *   ws            device, pm_select_workspace(alphabet, k, m, cap_buckets)
 *                 bytes, 8-byte aligned
 * The counts are read once.  Limit: |Sigma|^k <= 2^19 (PM_ERANGE above). */
int bucket_select(const pm_seqs *S, int32_t l, int32_t k, const uint32_t *keys,
                  const uint32_t *counts, int32_t m, uint32_t s, pm_bucket *buckets,
                  int64_t cap_buckets, uint32_t *members, int64_t cap_members, int64_t *n_out,
                  void *ws, size_t ws_bytes, uint32_t *status, void *stream);

/* a3 + a4 + a5 in one call -- projection_hash followed by bucket_select, with
 * the same keys, counts, buckets, members and n_out (bit for bit), but the
 * selection's passing-key bitmap and per-trial totals are formed by the hash
 * pass while each trial's histogram is still in LDS, so the counts are not
 * read back for them (Alg. 2 steps 2(b), 2(c) and 3; Sec. 6's bucket test,
 * a bucket passes with at least s l-mers, s = 0 as s = 1).
 *   keys, counts  device [m][x], [m][|Sigma|^k] uint32, both required
 *   masks         device [m]; a bad mask sets PM_STATUS_BAD_MASK and that
 *                 trial's keys and counts are not written and it gives no
 *                 buckets
 *   buckets, members, n_out, ws, truncation: as for bucket_select (ws:
 *                 pm_select_workspace(alphabet, k, m, cap_buckets) bytes,
 *                 8-byte aligned)
 * Limits: those of projection_hash and bucket_select (|Sigma|^k <= 2^19). */
int projection_hash_select(const pm_seqs *S, int32_t l, int32_t k, const uint32_t *masks, int32_t m,
                           uint32_t *keys, uint32_t *counts, uint32_t s, pm_bucket *buckets,
                           int64_t cap_buckets, uint32_t *members, int64_t cap_members, int64_t *n_out,
                           void *ws, size_t ws_bytes, uint32_t *status, void *stream);

/* a3 + a4 + a5 fused -- Alg. 2 steps 2(b), 2(c) and 3 without keys or counts
 * in device memory: each trial's histogram lives only in LDS, where its
 * passing bins (at least s l-mers, Sec. 6) are turned into bucket records and
 * member slots.  The outputs and their order are those of bucket_select
 * (buckets ascending by (trial, key), `first` and `size` identical) except
 * that the members of one bucket come in no particular order; n_out and
 * truncation as for bucket_select.  One call runs a counting pass, a scan and
 * the writing pass (with cap_buckets = cap_members = 0 only the first two,
 * to size the lists).
 *   masks   device [m] (bad masks: PM_STATUS_BAD_MASK, that trial contributes
 *           nothing)
 *   ws      device, pm_hash_select_workspace(S, l, k, m) bytes, 8-byte aligned;
 *           it starts with the number of enriched buckets of every (trial,
 *           key-range slice), trial-major (int64)
 * Limits: DNA k <= 16, protein k <= 7.  DNA k <= 12 and protein k <= 5 use
 * the LDS count table (sliced over workgroups when it does not fit one
 * workgroup's LDS); larger k use the sorted selection below, whose members
 * come in ascending window order. */
size_t pm_hash_select_workspace(const pm_seqs *S, int32_t l, int32_t k, int32_t m);
int bucket_hash_select(const pm_seqs *S, int32_t l, int32_t k, const uint32_t *masks, int32_t m, uint32_t s,
                       pm_bucket *buckets, int64_t cap_buckets, uint32_t *members, int64_t cap_members,
                       int64_t *n_out, void *ws, size_t ws_bytes, uint32_t *status, void *stream);

/* a3 + a4 + a5 for key spaces too large for a count table (the space
 * problem Sec. 6 answers with its K2 kernel and Fig. 8): the same bucket
 * list as bucket_select, formed by sorting each trial's (key, window) pairs
 * by key within key-range slices in LDS instead of counting into |Sigma|^k
 * bins.  Buckets ascending by (trial, key), members of each bucket in
 * ascending window order, `first` and `size` identical to bucket_select's;
 * n_out, truncation and bad masks as for bucket_hash_select (which calls this
 * path itself for DNA k > 12 and protein k > 5).
 *   ws   device, pm_sort_select_workspace(S, l, k, m) bytes, 8-byte aligned
 * Limits: DNA 8 <= k <= 16, protein 4 <= k <= 7 (PM_ERANGE otherwise). */
size_t pm_sort_select_workspace(const pm_seqs *S, int32_t l, int32_t k, int32_t m);
int bucket_sort_select(const pm_seqs *S, int32_t l, int32_t k, const uint32_t *masks, int32_t m, uint32_t s,
                       pm_bucket *buckets, int64_t cap_buckets, uint32_t *members, int64_t cap_members,
                       int64_t *n_out, void *ws, size_t ws_bytes, uint32_t *status, void *stream);

/* bucket_hash_select without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, outputs and order as
 * bucket_hash_select, minus ws/ws_bytes: the per-(trial, key-range slice)
 * totals and bases live in a fixed device array of
 * pm_hash_select_scratch_bytes() bytes (8 MiB) that each GPU holds from the
 * first call on it until the process ends.  A call whose trials x slices need
 * more (pm_hash_select_workspace() above that size, i.e. more than 262 136
 * trial-slices) returns PM_ERANGE before anything is enqueued.  Nothing
 * needs to start at zero: every call rewrites the entries it uses.  All calls
 * on one GPU share the array, so calls that overlap on that GPU (different
 * streams, or threads) race and must be serialised by the caller.  Allocates
 * nothing (no hipMalloc, hipFree or allocating library call). */
size_t pm_hash_select_scratch_bytes(void);
int bucket_hash_select_noalloc(const pm_seqs *S, int32_t l, int32_t k, const uint32_t *masks, int32_t m,
                               uint32_t s, pm_bucket *buckets, int64_t cap_buckets, uint32_t *members,
                               int64_t cap_members, int64_t *n_out, uint32_t *status, void *stream);

/* a6 (first half) -- Sec. 2 profile matrix P(s) of each bucket's alignment.
 *   members      device [cap_members] as written by bucket_select; a bucket
 *                whose members run past cap_members gets an all-zero profile
 *   B            host capacity (grid size); n_dev device count of valid
 *                buckets (e.g. n_out of bucket_select) or NULL when all B are
 *                valid
 *   profile      device [B][|Sigma|][l] uint32 letter counts per column */
int bucket_profile(const pm_seqs *S, int32_t l, const pm_bucket *buckets,
                   const uint32_t *members, int64_t cap_members, int64_t B, const int64_t *n_dev,
                   uint32_t *profile, void *stream);

/* a6 -- Sec. 5.1, Fig. 4: initial model theta^0 from the profile,
 * theta0 = (profile + beta * bg) / (size + beta) (beta = 0: the paper's raw
 * frequencies).  bg device [|Sigma|]; theta0 device [B][|Sigma|][l]. */
int theta_init(int32_t alphabet, int32_t l, const uint32_t *profile, int64_t B,
               const int64_t *n_dev, const double *bg, double beta, double *theta0, void *stream);

/* a7 - a10 -- Sec. 5.1, EM refinement of each model under the OOPS model
 * (Sec. 2).  The paper gives no formulas; the model is the standard OOPS EM
 * with a uniform start prior and fixed background bg:
 *   s_ia = sum_p ln(theta[S_i[a+p]][p] / bg[S_i[a+p]]),
 *   LSE_i = ln sum_a exp s_ia,  Z_ia = exp(s_ia - LSE_i),
 *   LLR = sum_i (LSE_i - ln L_i),  J = LLR + beta * sum bg ln theta,
 *   theta' = (sum Z_ia [S_i[a+p] = c] + beta * bg) / (t + beta).
 * `iters` M-steps, then a final E-step.
 *   theta0     device [B][|Sigma|][l]
 *   theta_out  device [B][|Sigma|][l]   (theta^iters)
 *   J_out      device [B][iters+1]      (J of theta^0 .. theta^iters)
 *   llr_out    device [B][iters+1] or NULL
 *   sites_out  device [B][t] int32 or NULL: argmax_a s_ia under theta^iters,
 *              first on ties
 *   precision  PM_FP64, PM_FP32, PM_F16X2 or PM_F16
 *   ws, ws_bytes  device workspace of at least pm_em_workspace(S, l, precision)
 *              bytes, 16-byte aligned, or NULL.  The DNA matrix-core forms keep
 *              the one-hot tables of every 32-window pair there (built once per
 *              call, read by every model); with NULL they rebuild them inside
 *              the EM kernel (same results, slower).  Other forms ignore it.
 *              A non-NULL workspace below the size is PM_EINVAL. */
int em_refine(const pm_seqs *S, int32_t l, const double *theta0, const double *bg, int64_t B,
              const int64_t *n_dev, int32_t iters, double beta, int32_t precision,
              double *theta_out, double *J_out, double *llr_out, int32_t *sites_out, void *ws,
              size_t ws_bytes, void *stream);

/* Sequence models of Sec. 2: OOPS (exactly one occurrence per sequence, the
 * model of em_refine), ZOOPS (zero or one) and TCM (zero or more). */
#define PM_OOPS 0
#define PM_ZOOPS 1
#define PM_TCM 2

/* a7 - a10 under ZOOPS or TCM (Sec. 2 defines both only in words; the
 * readings are the two-component mixtures of the MEME papers the paper
 * cites, with one mixing parameter `mix`):
 *   ZOOPS (mix = gamma, the probability that a sequence holds a site):
 *     LLR_i = ln((1 - gamma) + (gamma / L_i) sum_a e^{s_ia}),
 *     Z_ia = (gamma / L_i) e^{s_ia - LLR_i},  gamma' = sum Z / t;
 *   TCM (mix = lambda, the probability that a window is an occurrence,
 *     windows independent):
 *     LLR = sum_{i,a} ln((1 - lambda) + lambda e^{s_ia}),
 *     Z_ia = lambda e^{s_ia} / ((1 - lambda) + lambda e^{s_ia}),
 *     lambda' = sum Z / x;
 *   both: theta' = (sum Z_ia [S_i[a+p] = c] + beta * bg) / (sum Z + beta),
 *     J = LLR + beta * sum bg ln theta (never decreases), mix' capped at 1.
 * model PM_OOPS calls em_refine (mix0 ignored, mix_out not written).
 *   mix0      in (0, 1]; ZOOPS with gamma = 1 is OOPS
 *   mix_out   device [B] mixing parameter of the final E-step, or NULL
 *   sites_out device [B][t]: ZOOPS the best start of sequence i when its site
 *             mass sum_a Z_ia >= 1/2, TCM when that start's Z >= 1/2, else -1
 * Other arguments as em_refine; precision PM_FP64 or PM_FP32 (the vector
 * path), PM_EINVAL otherwise. */
int em_refine_model(const pm_seqs *S, int32_t l, int32_t model, double mix0, const double *theta0,
                    const double *bg, int64_t B, const int64_t *n_dev, int32_t iters, double beta,
                    int32_t precision, double *theta_out, double *mix_out, double *J_out, double *llr_out,
                    int32_t *sites_out, void *stream);
/* Gibbs site sampling as the local optimiser of each model, in place of EM
 * (Sec. 1 and Sec. 3 name Gibbs sampling beside EM; the site sampler of
 * Lawrence et al., cited by the paper).  Per model: start from the best start
 * of every sequence under theta0 (first on ties); each of `sweeps` sweeps
 * visits S_1..S_t in order and redraws S_i's start a with probability
 * proportional to prod_p theta[S_i[a+p]][p] / bg[S_i[a+p]], theta the
 * profile of the other t-1 sites with pseudocounts,
 * theta = (counts + beta * bg) / (t - 1 + beta) -- the draw is the first
 * start whose running weight sum exceeds u times the total;
 * u = (x >> 11) * 2^-53 with x the first word of Philox4x64-10 (Salmon et
 * al., SC'11) at key {seed, 0}, counter {sweep, i, model, 0}.  The answer is
 * the alignment of largest F = sum_{c,p} n_cp ln(theta_cp / bg_c) (n its
 * letter counts, theta = (n + beta * bg) / (t + beta)) among the start and
 * the end of every sweep, the earliest on ties.
 *   theta0     device [B][|Sigma|][l]
 *   theta_out  device [B][|Sigma|][l]: theta of the best alignment
 *   F_out      device [B][sweeps+1] (F of the start, then after each sweep), or NULL
 *   sites_out  device [B][t] best alignment's starts, or NULL
 * beta > 0 (PM_EINVAL otherwise); t <= 512 (PM_ERANGE).  FP64 throughout. */
int gibbs_refine(const pm_seqs *S, int32_t l, const double *theta0, const double *bg, int64_t B,
                 const int64_t *n_dev, int32_t sweeps, double beta, uint64_t seed, double *theta_out,
                 double *F_out, int32_t *sites_out, void *stream);

/* Workspace bytes of em_refine: the one-hot tables of the DNA matrix-core
 * forms (t + ceil(x/32) window pairs of 1 KB + (4 ceil(l/4) + 12) x 64 B each);
 * 0 for the other forms or invalid arguments. */
size_t pm_em_workspace(const pm_seqs *S, int32_t l, int32_t precision);

/* Tile-shape autotuner of the matrix-core EM (PM_F16X2, PM_F16): runs
 * em_refine on the caller's B models once per candidate shape, times each
 * with HIP events on `stream` (the call synchronises), and records the
 * fastest for models of length class ceil(l/4) and this precision in a
 * process-wide table that later em_refine / em_refine_batch calls use.
 * A shape is coded 10 G + PPB: G groups of 16 models per wave (1, or 2 for
 * l <= 24), PPB window pairs whose one-hot tables are staged per workgroup
 * barrier (1, 2 or 4).  Pass B of the size the later calls will have: the
 * shapes differ in workgroup size, so their ranking depends on how well B
 * fills the device.
 * theta_out, J_out: device scratch of em_refine's shapes (overwritten);
 * ws, ws_bytes: as for em_refine (pass the workspace the timed calls will
 * have).  DNA only.  choice_out: host int32[1] or NULL.  em_tuning returns
 * the shape in use (untuned: 14), or a negative status. */
int em_autotune(const pm_seqs *S, int32_t l, const double *theta0, const double *bg, int64_t B, int32_t iters,
                double beta, int32_t precision, double *theta_out, double *J_out, void *ws, size_t ws_bytes,
                int32_t *choice_out, void *stream);
int em_tuning(int32_t l, int32_t precision);
/* Records `shape` (coded as above) for l's length class and `precision`, in
 * place of a tuned or default one: for callers that tuned in an earlier
 * process or want a fixed shape.  PM_EINVAL for a shape the class cannot
 * take. */
int em_set_tuning(int32_t l, int32_t precision, int32_t shape);

/* a10 -- Sec. 5.1: the model with the highest objective wins.  best_out
 * device int64[1]: the bucket with the largest J(theta^iters), lowest index
 * on ties, -1 if none; consensus_out device char[l+1]: the letter of largest
 * probability per column of that model (lowest code on ties), NUL-ended. */
int em_best(const double *J, int64_t B, const int64_t *n_dev, int32_t iters, const double *theta,
            int32_t alphabet, int32_t l, int64_t *best_out, char *consensus_out, void *stream);

/* ---- Batches: many independent instances in one set of launches ----
 *
 * A batch holds P instances that share the alphabet, l and k (one shape
 * class); each has its own sequences (any t and n_i) and its own trials.  Trial items are numbered over the whole batch:
 * instance p owns items first_item .. first_item + m - 1, instances in item
 * order, so a bucket's `trial` field (the item) also names its instance.
 * Keys of item j of instance p sit at key_base + (j - first_item) * x in the
 * keys array, counts at j * |Sigma|^k; member numbers are window numbers
 * within the instance.  Every pass below is the single-instance call of the
 * same name run over all items, buckets or instances of the batch at once. */
typedef struct pm_inst {
    const int64_t *offsets;  /* device [t+1], as pm_seqs.offsets */
    const uint32_t *packed;  /* device, pm_pack words of this instance */
    int64_t n_total;         /* sum of the instance's n_i */
    int64_t x;               /* windows at the batch's l: n_total - t (l - 1) */
    int64_t key_base;        /* first key slot of the instance's first item */
    int32_t t;               /* sequences */
    int32_t n_min;           /* shortest sequence (>= l) */
    int32_t m;               /* trials (items) of the instance, >= 1 */
    int32_t first_item;      /* its first item */
} pm_inst;

typedef struct pm_batch {
    int32_t alphabet;          /* PM_DNA or PM_PROTEIN */
    int32_t l, k;              /* motif length and projection size of every instance */
    int32_t P;                 /* instances, >= 1 */
    int32_t items;             /* trial items: the sum of m */
    const pm_inst *inst;       /* device [P] */
    const pm_inst *inst_host;  /* host [P], the same contents (checks and launch sizes) */
    const int32_t *item_inst;  /* device [items]: the instance of every item */
} pm_batch;

/* Checks a batch's host table (item numbering, x, limits); PM_OK or PM_EINVAL. */
int pm_batch_check(const pm_batch *B);

/* a3 + a4 over every item of a batch.  masks device [items]; keys device
 * [sum_p m_p x_p] or NULL; counts device [items][|Sigma|^k] or NULL. */
int projection_hash_batch(const pm_batch *B, const uint32_t *masks, uint32_t *keys, uint32_t *counts,
                          uint32_t *status, void *stream);

/* a5 over every item of a batch; same outputs as bucket_select with `trial`
 * holding the item.  ws: pm_select_workspace(alphabet, k, items, cap_buckets)
 * bytes, 8-byte aligned. */
int bucket_select_batch(const pm_batch *B, const uint32_t *keys, const uint32_t *counts, uint32_t s,
                        pm_bucket *buckets, int64_t cap_buckets, uint32_t *members, int64_t cap_members,
                        int64_t *n_out, void *ws, size_t ws_bytes, uint32_t *status, void *stream);

/* projection_hash_select over every item of a batch: the outputs of
 * projection_hash_batch followed by bucket_select_batch.  ws:
 * pm_select_workspace(alphabet, k, items, cap_buckets) bytes, 8-byte aligned. */
int projection_hash_select_batch(const pm_batch *B, const uint32_t *masks, uint32_t *keys, uint32_t *counts,
                                 uint32_t s, pm_bucket *buckets, int64_t cap_buckets, uint32_t *members,
                                 int64_t cap_members, int64_t *n_out, void *ws, size_t ws_bytes,
                                 uint32_t *status, void *stream);

/* The fused a3 - a5 over every item of a batch (bucket `trial` = item);
 * ws: pm_hash_select_batch_workspace(B) bytes. */
size_t pm_hash_select_batch_workspace(const pm_batch *B);
int bucket_hash_select_batch(const pm_batch *B, const uint32_t *masks, uint32_t s, pm_bucket *buckets,
                             int64_t cap_buckets, uint32_t *members, int64_t cap_members, int64_t *n_out, void *ws,
                             size_t ws_bytes, uint32_t *status, void *stream);
/* bucket_sort_select over a batch (trial = item number, as above).
 *   ws  device, pm_sort_select_batch_workspace(B) bytes, 8-byte aligned */
size_t pm_sort_select_batch_workspace(const pm_batch *B);
int bucket_sort_select_batch(const pm_batch *B, const uint32_t *masks, uint32_t s, pm_bucket *buckets,
                             int64_t cap_buckets, uint32_t *members, int64_t cap_members, int64_t *n_out,
                             void *ws, size_t ws_bytes, uint32_t *status, void *stream);

/* a6 (profiles) for the buckets of a batch. */
int bucket_profile_batch(const pm_batch *B, const pm_bucket *buckets, const uint32_t *members,
                         int64_t cap_members, int64_t Bcap, const int64_t *n_dev, uint32_t *profile,
                         void *stream);

/* Workspace bytes em_refine_batch needs for batch B in `precision`: for the
 * DNA matrix-core forms the workgroup plan, every instance's first table slot
 * and the one-hot tables of all its window pairs (as for em_refine); 0 for the
 * vector forms (no workspace) or an invalid batch. */
size_t pm_em_batch_workspace(const pm_batch *B, int32_t precision);

/* a7 - a10 for every bucket of a batch, each against its own instance
 * (buckets as written by bucket_select_batch, ascending by item).  sites_out
 * is [Bcap][t_max] with t_max the largest t of the batch (entries past the
 * instance's t untouched).  The matrix-core form groups the buckets of one
 * instance into workgroups and issues the instances largest first; it needs
 * ws of pm_em_batch_workspace(B, precision) bytes, 256-byte aligned
 * (PM_EINVAL otherwise). */
int em_refine_batch(const pm_batch *B, const pm_bucket *buckets, const double *theta0, const double *bg,
                    int64_t Bcap, const int64_t *n_dev, int32_t iters, double beta, int32_t precision,
                    double *theta_out, double *J_out, double *llr_out, int32_t *sites_out, void *ws,
                    size_t ws_bytes, void *stream);

/* a10 per instance: best_out device int64[P] (bucket index or -1),
 * consensus_out device char[P][l+1]. */
int em_best_batch(const pm_batch *B, const pm_bucket *buckets, const double *J, int64_t Bcap,
                  const int64_t *n_dev, int32_t iters, const double *theta, int64_t *best_out,
                  char *consensus_out, void *stream);

/* ---- Learned bucket triage ----
 *
 * An addition to the paper's method, which refines every enriched bucket
 * (Sec. 5.1): a small network scores every bucket from its profile, EM refines
 * only the best-scored fraction of each instance, and an instance whose refined
 * winner does not stand out from the other refined buckets (a z-score of its
 * objective below a threshold) has all its other buckets refined too.  DNA
 * only, l <= 21.
 *
 * Network: 87 inputs -> 256 -> 256 -> 1, ReLU after both hidden layers.  FP32
 * parameters in one flat vector of PM_TRIAGE_PARAMS floats:
 *   W1 [87][256], b1 [256], W2 [256][256], b2 [256], w3 [256][1], b3 [1]
 * (W[i][o]: input i to output o).  Inputs of a bucket (feature index):
 *   4r + j (r < 21, j < 4)  the j-th largest letter frequency (profile / size)
 *                           of the r-th column, columns in decreasing
 *                           lexicographic order of their sorted counts; 0 for
 *                           r >= l (which letters and positions agree says
 *                           nothing of a motif: the projection is random)
 *   84  ln(size); 85  background entropy in bits; 86  the largest column
 *   information content in bits, sum_c f log2(f / bg_c)
 * each optionally standardised, (v - mu[i]) / sd[i]. */
#define PM_TRIAGE_PARAMS 88577
#define PM_TRIAGE_INPUTS 87

/* Features of B buckets from their profiles (bucket_profile layout, DNA).
 * bg device [4]; mu, sd device [87] or both NULL (raw features);
 * feat device [B][87] FP32. */
int triage_features(int32_t l, const uint32_t *profile, int64_t B, const int64_t *n_dev, const double *bg,
                    const float *mu, const float *sd, float *feat, void *stream);

/* Serving weights: BF16 matrix-core fragments of W1 and W2 plus FP32 biases
 * and w3, pm_triage_packed_bytes() bytes of device memory, from the FP32
 * parameter vector (device). */
size_t pm_triage_packed_bytes(void);
int triage_pack(const float *params, void *packed, void *stream);

/* Scores of B buckets: BF16 inputs, weights and first hidden layer, FP32
 * accumulation and second layer.  feat device [B][87]; score device [B]. */
int triage_forward(const void *packed, const float *feat, int64_t B, const int64_t *n_dev, float *score,
                   void *stream);

/* One training step on N examples, all in FP32: forward, mean squared error
 * against target, backward by the chain rule and, when lr > 0, one Adam
 * update (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected; step counts from
 * 1).  params, adam_m, adam_v device [PM_TRIAGE_PARAMS]; X device [N][87];
 * target device [N]; loss_out device float[1] or NULL; grads_out device
 * [PM_TRIAGE_PARAMS] or NULL (else kept in ws); ws pm_triage_workspace(N)
 * bytes. */
size_t pm_triage_workspace(int32_t N);
int triage_train_step(float *params, float *adam_m, float *adam_v, int32_t step, const float *X,
                      const float *target, int32_t N, float lr, float *loss_out, float *grads_out, void *ws,
                      size_t ws_bytes, void *stream);

/* Per instance (Bt: a batch, buckets ascending by item; NULL: the B buckets
 * of one instance), keep every bucket whose score is at least the c-th
 * largest score of the instance, c = max(1, ceil(frac n_instance)) (ties all
 * kept), and compact the kept buckets, in order, with their theta^0 rows.
 *   taken       device uint8 [B] or NULL: set to 1 for kept buckets (cleared first)
 *   sel_buckets device [B], sel_theta0 device [B][|Sigma|][l],
 *   sel_index   device int64 [B] or NULL: original index of each kept bucket
 *   n_sel       device int64[1]: number kept
 *   ws          pm_triage_select_workspace(P, B) bytes, kept for the fallback */
size_t pm_triage_select_workspace(int32_t P, int64_t B);
int triage_select(const pm_batch *Bt, const pm_bucket *buckets, const float *score, int64_t B,
                  const int64_t *n_dev, double frac, const double *theta0, int32_t alphabet, int32_t l,
                  uint8_t *taken, pm_bucket *sel_buckets, double *sel_theta0, int64_t *sel_index,
                  int64_t *n_sel, void *ws, size_t ws_bytes, void *stream);

/* Fallback after EM of the triaged buckets (list 1: sel1 / n_sel1 as written
 * by triage_select, best device int64 [P] and J device [n_sel1][iters+1] from
 * em_best / em_best_batch and em_refine on it).  Per instance, z = (J_w - mean)
 * / sd of the winner's J(theta^iters) among the J of every bucket of the
 * instance in list 1 (0 when sd = 0, -inf without a winner); an instance with
 * z below `threshold` gets all its buckets not taken by triage_select
 * compacted as above.  fell_back device int32 [P] or NULL; z_out device
 * double [P] or NULL.  Same ws as the preceding triage_select. */
int triage_fallback_select(const pm_batch *Bt, const pm_bucket *buckets, int64_t B, const int64_t *n_dev,
                           const pm_bucket *sel1, const int64_t *n_sel1, const int64_t *best, const double *J,
                           int32_t iters, double threshold, const double *theta0, int32_t alphabet, int32_t l,
                           uint8_t *taken, pm_bucket *sel_buckets, double *sel_theta0, int64_t *sel_index,
                           int64_t *n_sel, int32_t *fell_back, double *z_out, void *ws, size_t ws_bytes,
                           void *stream);

/* Per instance, the better of the triaged winner (list 1) and the fallback
 * winner (list 2, or best2 NULL): larger J(theta^iters), lower original bucket
 * index on ties.  best_out device int64 [P]: original bucket index or -1;
 * consensus_out device char [P][l+1] or NULL. */
int triage_merge_best(int32_t P, int32_t alphabet, int32_t l, int32_t iters, const int64_t *best1,
                      const int64_t *index1, const double *J1, const double *theta1, const int64_t *best2,
                      const int64_t *index2, const double *J2, const double *theta2, int64_t *best_out,
                      char *consensus_out, void *stream);

/* ---- The whole path, host in, host out (Alg. 2 and Alg. 3 INPUT/OUTPUT) ---- */
typedef struct pm_problem {
    int32_t alphabet;          /* PM_DNA or PM_PROTEIN */
    int32_t t;                 /* number of sequences S_1..S_t */
    const char *const *seqs;   /* host [t] strings (need not be NUL-ended) */
    const int32_t *n;          /* host [t] lengths, each >= l */
    int32_t l, d;              /* motif length, mutations (d only feeds the automatic parameters) */
    int32_t k, s, m;           /* projection size, threshold, trials; <= 0: chosen by
                                  pm_auto_params (Sec. 5) */
    const uint32_t *masks;     /* host [m] or NULL: drawn by pm_masks_from_seed(seed);
                                  when given, m must be their number */
    uint64_t seed;
    const double *bg;          /* host [|Sigma|] in code order (normalised here), or NULL:
                                  the composition of the input (every letter must occur) */
} pm_problem;

typedef struct pm_options {
    int32_t em_iters;          /* M-steps per model (then a final E-step) */
    double beta;               /* pseudocount mass for theta^0 and the M-step */
    int32_t precision;         /* PM_FP64, PM_FP32, PM_F16X2 or PM_F16 (protein PM_F16 only with
                                  batched = 0 and triage = 0) */
    int32_t batched;           /* 0: problems one after another through the single-instance
                                  calls; 1: problems sharing alphabet, l, k, s and background run
                                  as one batch each (projection_hash_batch ... em_best_batch) */
    int32_t triage;            /* 1: learned bucket triage (DNA, l <= 21): EM of the
                                  triage_frac best-scored buckets of each problem, fallback to all
                                  its other buckets when the winner is weak, better winner kept */
    double triage_frac;        /* fraction refined first; <= 0 means 0.05 */
    const char *triage_weights;/* path of a weights file (format below); required with triage */
    void *stream;              /* hipStream_t or NULL */
} pm_options;

/* Triage weights file, little-endian: the 8 bytes "PMTRIAG1"; int32
 * PM_TRIAGE_PARAMS; int32 PM_TRIAGE_INPUTS; float params[PM_TRIAGE_PARAMS]
 * (layout as for triage_train_step); float mu[PM_TRIAGE_INPUTS]; float
 * sd[PM_TRIAGE_INPUTS]; double pooled fallback threshold; int32 n; then n
 * records {int32 l; double threshold} of per-motif-length thresholds. */

typedef struct pm_result {
    char *consensus;           /* host [l+1], caller-owned, or NULL; "" when nothing was enriched */
    int32_t *sites;            /* host [t], caller-owned, or NULL: 0-based starts */
    double *theta;             /* host [|Sigma|][l], caller-owned, or NULL */
    double J, llr;             /* objective and log-likelihood ratio of the answer (-inf: none) */
    int32_t best_trial;        /* trial of the winning bucket within its problem, -1: none */
    uint32_t best_key;
    int64_t n_enriched;        /* enriched buckets of the problem */
    int64_t n_refined;         /* buckets refined by EM (all of them without triage) */
    int32_t fallback_used;     /* 1 when triage fell back to refining the problem's other buckets */
    int32_t k, s, m;           /* parameters used */
} pm_result;

/* Runs n_problems problems (R[p] answers P[p]); synchronous at return.  This
 * convenience entry point allocates and frees its own device buffers.
 * PM_EINVAL names the problem at fault in pm_last_error(). */
int projection_run(const pm_problem *P, int32_t n_problems, const pm_options *O, pm_result *R);

/* A motif-length range (l-, l+) (Sec. 2): the problem P run at every length
 * l- .. l+ in one projection_run call (P->l ignored; k, s, m <= 0 chosen per
 * length by pm_auto_params from P->d, a given k must not exceed l-; masks
 * must be NULL, drawn per length from P->seed).  R[q] (host [l+ - l- + 1],
 * consensus buffers of l- + q + 1 bytes) answers length l- + q.  *chosen (or
 * NULL) receives the length whose answer has the largest LLR per motif column
 * (the longer on ties; the paper does not say how lengths compete), -1 when
 * no length has an enriched bucket. */
int projection_run_range(const pm_problem *P, int32_t l_minus, int32_t l_plus, const pm_options *O, pm_result *R,
                         int32_t *chosen);

#ifdef __cplusplus
}
#endif

#endif /* PROJMOTIF_H */
