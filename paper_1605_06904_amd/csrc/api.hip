// Host side of libprojmotif: error reporting, argument checks and the
// host-side parameter helpers (Sec. 5 and Sec. 6 of the paper).
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
