// Host side of libprojmotif: error reporting, argument checks, host-side
// parameter helpers (Sec. 5 and Sec. 6 of the paper) and projection_run, the
// host-in/host-out driver of the whole path.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "pm_common.h"

namespace pm {

static thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

void clear_error() { g_err.clear(); }

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

int device_lds_bytes()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 64 * 1024;
    static int cached[64] = {0};
    if (dev >= 0 && dev < 64 && cached[dev]) return cached[dev];
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
        v = 64 * 1024;
    if (dev >= 0 && dev < 64) cached[dev] = v;
    return v;
}

int check_seqs(const pm_seqs *S, int l)
{
    if (!S) return fail(PM_EINVAL, "sequences are NULL");
    if (S->alphabet != 4 && S->alphabet != 20) return fail(PM_EINVAL, "alphabet must be 4 or 20");
    if (S->t < 1) return fail(PM_EINVAL, "need t >= 1 sequences");
    if (!S->offsets || !S->packed) return fail(PM_EINVAL, "offsets/packed are NULL");
    if (l < 1 || l > 32) return fail(PM_EINVAL, "need 1 <= l <= 32 (l=%d)", l);
    if (S->n_min < l) return fail(PM_EINVAL, "every sequence must be at least l=%d long (n_min=%d)", l, S->n_min);
    if (S->n_max < S->n_min || S->n_total < (int64_t)S->n_min * S->t || S->n_total > (int64_t)S->n_max * S->t)
        return fail(PM_EINVAL, "inconsistent n_total/n_min/n_max");
    if (S->n_total >= (1ll << 31)) return fail(PM_ERANGE, "n_total must stay below 2^31");
    return PM_OK;
}

pm_inst inst_of(const pm_seqs *S, int l)
{
    pm_inst I{};
    I.offsets = S->offsets;
    I.packed = S->packed;
    I.n_total = S->n_total;
    I.x = num_windows(S, l);
    I.key_base = 0;
    I.t = S->t;
    I.n_min = S->n_min;
    I.m = 0;
    I.first_item = 0;
    return I;
}

int check_batch(const pm_batch *B, BatchInfo *info)
{
    if (!B) return fail(PM_EINVAL, "batch is NULL");
    if (B->alphabet != 4 && B->alphabet != 20) return fail(PM_EINVAL, "alphabet must be 4 or 20");
    if (B->l < 1 || B->l > 32) return fail(PM_EINVAL, "need 1 <= l <= 32 (l=%d)", B->l);
    if (B->k < 1 || B->k > B->l) return fail(PM_EINVAL, "need 1 <= k <= l (k=%d, l=%d)", B->k, B->l);
    if (B->P < 1 || B->items < 1) return fail(PM_EINVAL, "need P >= 1 and items >= 1");
    if (!B->inst || !B->inst_host || !B->item_inst) return fail(PM_EINVAL, "batch tables are NULL");
    BatchInfo in{};
    int64_t item = 0, key = 0;
    for (int p = 0; p < B->P; ++p) {
        const pm_inst &I = B->inst_host[p];
        if (I.t < 1 || !I.offsets || !I.packed) return fail(PM_EINVAL, "instance %d: bad sequences", p);
        if (I.n_min < B->l) return fail(PM_EINVAL, "instance %d: a sequence is shorter than l", p);
        if (I.n_total < (int64_t)I.n_min * I.t || I.n_total >= (1ll << 31))
            return fail(PM_EINVAL, "instance %d: bad n_total", p);
        if (I.x != I.n_total - (int64_t)I.t * (B->l - 1)) return fail(PM_EINVAL, "instance %d: x != n_total - t (l - 1)", p);
        if (I.m < 1) return fail(PM_EINVAL, "instance %d: m must be >= 1", p);
        if (I.first_item != item) return fail(PM_EINVAL, "instance %d: first_item must be %lld", p, (long long)item);
        if (I.key_base != key) return fail(PM_EINVAL, "instance %d: key_base must be %lld", p, (long long)key);
        item += I.m;
        key += (int64_t)I.m * I.x;
        in.t_max = std::max(in.t_max, I.t);
        in.nw_max = std::max<int64_t>(in.nw_max, pm_packed_words(B->alphabet, I.n_total));
        in.x_max = std::max(in.x_max, I.x);
    }
    if (item != B->items) return fail(PM_EINVAL, "items (%d) is not the sum of m (%lld)", B->items, (long long)item);
    in.keys_total = key;
    if (info) *info = in;
    return PM_OK;
}

}  // namespace pm

using namespace pm;

extern "C" int pm_batch_check(const pm_batch *B)
{
    clear_error();
    return check_batch(B, nullptr);
}

extern "C" const char *pm_version(void) { return "projmotif 0.1 (gfx950)"; }

extern "C" const char *pm_last_error(void) { return g_err.c_str(); }

// Park-Miller minimal standard generator, x <- 16807 x mod (2^31 - 1).
static uint32_t parkmiller_next(uint64_t *st)
{
    *st = (*st * 16807ull) % 2147483647ull;
    return (uint32_t)*st;
}

extern "C" int pm_masks_from_seed(uint64_t seed, int32_t l, int32_t k, int32_t m, uint32_t *masks)
{
    clear_error();
    if (l < 1 || l > 32 || k < 1 || k > l || m < 0) return fail(PM_EINVAL, "need 1 <= k <= l <= 32, m >= 0");
    if (m > 0 && !masks) return fail(PM_EINVAL, "masks is NULL");
    for (int32_t j = 0; j < m; ++j) {
        uint64_t st = 1 + (seed + (uint64_t)j) % 2147483646ull;
        int perm[32];
        for (int p = 0; p < l; ++p) perm[p] = p;
        uint32_t mask = l == 32 ? 0xffffffffu : ((1u << l) - 1u);
        // the first l-k entries of a partial shuffle are the positions left out
        for (int i = 0; i < l - k; ++i) {
            const int r = i + (int)(parkmiller_next(&st) % (uint32_t)(l - i));
            const int tmp = perm[i];
            perm[i] = perm[r];
            perm[r] = tmp;
            mask &= ~(1u << perm[i]);
        }
        masks[j] = mask;
    }
    return PM_OK;
}

static double binom_at_least(int t, double p, int s)
{
    // P[Binomial(t, p) >= s] = 1 - B(s), summed term by term in log space, so
    // that log B = log1p(-tail) keeps its precision when B is close to 1
    double acc = 0;
    for (int i = s < 0 ? 0 : s; i <= t; ++i) {
        const double lc = lgamma(t + 1.0) - lgamma(i + 1.0) - lgamma(t - i + 1.0);
        const double term = (p <= 0) ? (i == 0 ? 1.0 : 0.0)
                          : (p >= 1) ? (i == t ? 1.0 : 0.0)
                                     : exp(lc + i * log(p) + (t - i) * log1p(-p));
        acc += term;
    }
    return acc;
}

extern "C" int pm_auto_params(int32_t alphabet, int32_t t, int64_t x, int32_t l, int32_t d, double q,
                              int32_t *k, int32_t *s, int32_t *m)
{
    clear_error();
    if ((alphabet != 4 && alphabet != 20) || t < 1 || x < 1 || l < 2 || d < 0 || d >= l - 1 || !(q > 0 && q < 1))
        return fail(PM_EINVAL, "bad arguments to pm_auto_params");
    const int kk = l - d - 1;
    const double mean = (double)x / pow((double)alphabet, kk);
    const double s2 = ceil(2.0 * mean);
    const int ss = s2 < 3 ? 3 : (s2 > t ? t + 1 : (int)s2);
    if (ss > t) return fail(PM_ERANGE, "threshold s=%.0f exceeds t=%d: the planted bucket cannot pass", s2, t);
    // p_hat = C(l-d, k) / C(l, k)
    const double lp = lgamma(l - d + 1.0) - lgamma(kk + 1.0) - lgamma(l - d - kk + 1.0) -
                      (lgamma(l + 1.0) - lgamma(kk + 1.0) - lgamma(l - kk + 1.0));
    const double tail = binom_at_least(t, exp(lp), ss);
    double mm_d = 1;
    if (tail > 0 && tail < 1) mm_d = ceil(log(1 - q) / log1p(-tail));
    else if (tail <= 0) return fail(PM_ERANGE, "the planted bucket can never reach s=%d", ss);
    if (!(mm_d < 2147483647.0)) return fail(PM_ERANGE, "m would exceed 2^31 - 1");
    const int mm = mm_d < 1 ? 1 : (int)mm_d;
    if (k) *k = kk;
    if (s) *s = ss;
    if (m) *m = mm;
    return PM_OK;
}

namespace {

struct DevBuf {
    void *p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
    int alloc(size_t n)
    {
        if (p) {
            (void)hipFree(p);
            p = nullptr;
        }
        if (n == 0) n = 16;
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) return fail(PM_EDEVICE, "hipMalloc(%zu) failed: %s", n, hipGetErrorString(e));
        return PM_OK;
    }
    template <typename T>
    T *as() const { return static_cast<T *>(p); }
};

}  // namespace

#define PM_CALL(expr)       \
    do {                    \
        int rc_ = (expr);   \
        if (rc_) return rc_; \
    } while (0)

extern "C" int projection_run(const pm_problem *P, const pm_options *O, pm_result *R)
{
    clear_error();
    if (!P || !O || !R) return fail(PM_EINVAL, "NULL argument");
    const int A = P->alphabet;
    if (A != 4 && A != 20) return fail(PM_EINVAL, "alphabet must be 4 or 20");
    if (P->t < 1 || !P->seqs || !P->n) return fail(PM_EINVAL, "need t >= 1 sequences");
    const int l = P->l;
    int64_t n_total = 0;
    int n_min = 0x7fffffff, n_max = 0;
    for (int i = 0; i < P->t; ++i) {
        if (!P->seqs[i] || P->n[i] < 0) return fail(PM_EINVAL, "sequence %d is NULL or has negative length", i);
        n_total += P->n[i];
        n_min = P->n[i] < n_min ? P->n[i] : n_min;
        n_max = P->n[i] > n_max ? P->n[i] : n_max;
    }
    if (l < 1 || l > 32 || n_min < l) return fail(PM_EINVAL, "need 1 <= l <= 32 and l <= every n_i");
    const int64_t x = n_total - (int64_t)P->t * (l - 1);
    int k = P->k, s = P->s, m = P->m;
    if (k <= 0 || s <= 0 || m <= 0) {
        int ak, as, am;
        PM_CALL(pm_auto_params(A, P->t, x, l, P->d, 0.95, &ak, &as, &am));
        if (k <= 0) k = ak;
        if (s <= 0) s = as;
        if (m <= 0) m = am;
    }
    if (k < 1 || k > l) return fail(PM_EINVAL, "need 1 <= k <= l");
    if (O->em_iters < 0 || O->beta < 0) return fail(PM_EINVAL, "need em_iters >= 0 and beta >= 0");
    hipStream_t st = as_stream(O->stream);

    // host staging: concatenated ASCII, offsets, masks, background
    std::vector<uint8_t> ascii((size_t)n_total);
    std::vector<int64_t> off(P->t + 1, 0);
    for (int i = 0; i < P->t; ++i) {
        memcpy(ascii.data() + off[i], P->seqs[i], (size_t)P->n[i]);
        off[i + 1] = off[i] + P->n[i];
    }
    std::vector<uint32_t> masks((size_t)m);
    if (P->masks) memcpy(masks.data(), P->masks, sizeof(uint32_t) * m);
    else PM_CALL(pm_masks_from_seed(P->seed, l, k, m, masks.data()));
    for (int j = 0; j < m; ++j)
        if (__builtin_popcount(masks[j]) != k || (l < 32 && (masks[j] >> l)))
            return fail(PM_EINVAL, "mask %d does not keep exactly k=%d of l=%d positions", j, k, l);

    const int64_t nw = pm_packed_words(A, n_total);
    const int64_t nb = ipow(A, k);
    DevBuf d_ascii, d_off, d_packed, d_masks, d_keys, d_counts, d_status, d_nout, d_ws;
    PM_CALL(d_ascii.alloc(n_total));
    PM_CALL(d_off.alloc(sizeof(int64_t) * (P->t + 1)));
    PM_CALL(d_packed.alloc(sizeof(uint32_t) * nw));
    PM_CALL(d_masks.alloc(sizeof(uint32_t) * m));
    PM_CALL(d_keys.alloc(sizeof(uint32_t) * (size_t)m * x));
    PM_CALL(d_counts.alloc(sizeof(uint32_t) * (size_t)m * nb));
    PM_CALL(d_status.alloc(sizeof(uint32_t)));
    PM_CALL(d_nout.alloc(sizeof(int64_t) * 2));
    PM_TRY(hipMemcpyAsync(d_ascii.p, ascii.data(), n_total, hipMemcpyHostToDevice, st));
    PM_TRY(hipMemcpyAsync(d_off.p, off.data(), sizeof(int64_t) * (P->t + 1), hipMemcpyHostToDevice, st));
    PM_TRY(hipMemcpyAsync(d_masks.p, masks.data(), sizeof(uint32_t) * m, hipMemcpyHostToDevice, st));
    PM_TRY(hipMemsetAsync(d_status.p, 0, sizeof(uint32_t), st));

    pm_seqs S{A, P->t, n_total, n_min, n_max, d_off.as<int64_t>(), d_packed.as<uint32_t>()};
    PM_CALL(pm_pack(A, d_ascii.as<uint8_t>(), n_total, d_packed.as<uint32_t>(), d_status.as<uint32_t>(), st));
    PM_CALL(projection_hash(&S, l, k, d_masks.as<uint32_t>(), m, d_keys.as<uint32_t>(),
                            d_counts.as<uint32_t>(), d_status.as<uint32_t>(), st));
    // size the bucket lists: one selection pass with empty capacities
    PM_CALL(d_ws.alloc(pm_select_workspace(m, 0)));
    PM_CALL(bucket_select(&S, l, k, d_keys.as<uint32_t>(), d_counts.as<uint32_t>(), m, (uint32_t)s, nullptr, 0,
                          nullptr, 0, d_nout.as<int64_t>(), d_ws.p, pm_select_workspace(m, 0), nullptr, st));
    int64_t nout[2];
    uint32_t status = 0;
    PM_TRY(hipMemcpyAsync(nout, d_nout.p, sizeof(nout), hipMemcpyDeviceToHost, st));
    PM_TRY(hipMemcpyAsync(&status, d_status.p, sizeof(status), hipMemcpyDeviceToHost, st));
    PM_TRY(hipStreamSynchronize(st));
    if (status & PM_STATUS_BAD_SYMBOL) return fail(PM_EINVAL, "a sequence holds a symbol outside the alphabet");
    if (status & PM_STATUS_BAD_MASK) return fail(PM_EINVAL, "bad projection mask");
    const int64_t nbk = nout[0], nmem = nout[1];
    R->k = k;
    R->s = s;
    R->m = m;
    R->n_enriched = nbk;
    R->best_trial = -1;
    R->best_key = 0;
    R->J = R->llr = -INFINITY;
    if (nbk == 0) {
        if (R->consensus) R->consensus[0] = 0;
        return PM_OK;
    }
    DevBuf d_bk, d_mem, d_prof, d_bg, d_th0, d_th, d_J, d_llr, d_sites, d_best, d_cons, d_emws;
    PM_CALL(d_bk.alloc(sizeof(pm_bucket) * nbk));
    PM_CALL(d_mem.alloc(sizeof(uint32_t) * nmem));
    PM_CALL(d_ws.alloc(pm_select_workspace(m, nbk)));
    PM_CALL(bucket_select(&S, l, k, d_keys.as<uint32_t>(), d_counts.as<uint32_t>(), m, (uint32_t)s,
                          d_bk.as<pm_bucket>(), nbk, d_mem.as<uint32_t>(), nmem, d_nout.as<int64_t>(), d_ws.p,
                          pm_select_workspace(m, nbk), d_status.as<uint32_t>(), st));
    // keys and counts are no longer needed
    (void)hipFree(d_keys.p);
    d_keys.p = nullptr;
    (void)hipFree(d_counts.p);
    d_counts.p = nullptr;

    std::vector<double> bg(A, 0.0);
    if (P->bg) {
        double tot = 0;
        for (int c = 0; c < A; ++c) tot += P->bg[c];
        for (int c = 0; c < A; ++c) bg[c] = P->bg[c] / tot;
    } else {
        // composition of the input (the background is fixed, never re-estimated)
        std::vector<double> cnt(A, 0.0);
        for (int64_t g = 0; g < n_total; ++g) {
            const char ch = (char)ascii[g];
            const char u = (ch >= 'a' && ch <= 'z') ? (char)(ch - 'a' + 'A') : ch;
            const char *L = A == 4 ? "ACTG" : "ARNDCQEGHILKMFPSTWYV";
            const char *f = strchr(L, u);
            if (f && u) cnt[f - L] += 1;
        }
        for (int c = 0; c < A; ++c) bg[c] = cnt[c] / (double)n_total;
    }
    const int AL = A * l;
    const int it1 = O->em_iters + 1;
    PM_CALL(d_prof.alloc(sizeof(uint32_t) * nbk * AL));
    PM_CALL(d_bg.alloc(sizeof(double) * A));
    PM_CALL(d_th0.alloc(sizeof(double) * nbk * AL));
    PM_CALL(d_th.alloc(sizeof(double) * nbk * AL));
    PM_CALL(d_J.alloc(sizeof(double) * nbk * it1));
    PM_CALL(d_llr.alloc(sizeof(double) * nbk * it1));
    PM_CALL(d_sites.alloc(sizeof(int32_t) * nbk * P->t));
    PM_CALL(d_best.alloc(sizeof(int64_t)));
    PM_CALL(d_cons.alloc(l + 1));
    const size_t em_ws = pm_em_workspace(&S, l, O->precision);
    if (em_ws) PM_CALL(d_emws.alloc(em_ws));
    PM_TRY(hipMemcpyAsync(d_bg.p, bg.data(), sizeof(double) * A, hipMemcpyHostToDevice, st));
    PM_CALL(bucket_profile(&S, l, d_bk.as<pm_bucket>(), d_mem.as<uint32_t>(), nmem, nbk, nullptr,
                           d_prof.as<uint32_t>(), st));
    PM_CALL(theta_init(A, l, d_prof.as<uint32_t>(), nbk, nullptr, d_bg.as<double>(), O->beta, d_th0.as<double>(), st));
    PM_CALL(em_refine(&S, l, d_th0.as<double>(), d_bg.as<double>(), nbk, nullptr, O->em_iters, O->beta,
                      O->precision, d_th.as<double>(), d_J.as<double>(), d_llr.as<double>(),
                      d_sites.as<int32_t>(), d_emws.p, em_ws, st));
    PM_CALL(em_best(d_J.as<double>(), nbk, nullptr, O->em_iters, d_th.as<double>(), A, l, d_best.as<int64_t>(),
                    d_cons.as<char>(), st));
    int64_t best = -1;
    PM_TRY(hipMemcpyAsync(&best, d_best.p, sizeof(best), hipMemcpyDeviceToHost, st));
    PM_TRY(hipStreamSynchronize(st));
    if (best < 0) {
        if (R->consensus) R->consensus[0] = 0;
        return PM_OK;
    }
    pm_bucket bk;
    PM_TRY(hipMemcpyAsync(&bk, d_bk.as<pm_bucket>() + best, sizeof(bk), hipMemcpyDeviceToHost, st));
    PM_TRY(hipMemcpyAsync(&R->J, d_J.as<double>() + best * it1 + O->em_iters, sizeof(double), hipMemcpyDeviceToHost, st));
    PM_TRY(hipMemcpyAsync(&R->llr, d_llr.as<double>() + best * it1 + O->em_iters, sizeof(double), hipMemcpyDeviceToHost, st));
    if (R->consensus) PM_TRY(hipMemcpyAsync(R->consensus, d_cons.p, l + 1, hipMemcpyDeviceToHost, st));
    if (R->sites)
        PM_TRY(hipMemcpyAsync(R->sites, d_sites.as<int32_t>() + best * P->t, sizeof(int32_t) * P->t,
                              hipMemcpyDeviceToHost, st));
    if (R->theta)
        PM_TRY(hipMemcpyAsync(R->theta, d_th.as<double>() + best * AL, sizeof(double) * AL, hipMemcpyDeviceToHost, st));
    PM_TRY(hipStreamSynchronize(st));
    R->best_trial = (int32_t)bk.trial;
    R->best_key = bk.key;
    return PM_OK;
}
