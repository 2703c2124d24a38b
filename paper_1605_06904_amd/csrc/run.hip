// projection_run: the whole path over one or many problems, host in, host
// out (the INPUT and OUTPUT of Alg. 2 and Alg. 3 of the paper).
//
// Each problem is validated and its parameters completed on the host (k, s
// and m from Sec. 5 when not given, masks from the seeded Park-Miller tables
// of Sec. 6 when not given, the background from the input composition when
// not given).  Problems then run either one after another through the
// single-instance entry points, or, batched, as one set of launches per
// group of problems that share the alphabet, l, k, s and background: every
// instance's ASCII is padded to whole packed words so that one pm_pack gives
// each its own region, and the batch entry points hash, select, profile,
// refine and pick the best of all of them at once.  With learned triage a
// network scores every bucket, EM refines the best-scored fraction of each
// instance, instances whose winner is weak fall back to refining the rest,
// and the better winner is kept (the same calls, in the same order, as the
// binding's triaged batch pipeline).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "pm_common.h"

namespace pm {
namespace {

struct DevBuf {
    void *p = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
    }
    int alloc(size_t n)
    {
        release();
        if (n == 0) n = 16;
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) return fail(PM_EDEVICE, "hipMalloc(%zu) failed: %s", n, hipGetErrorString(e));
        return PM_OK;
    }
    template <typename T>
    T *as() const { return static_cast<T *>(p); }
};

#define PM_CALL(expr)        \
    do {                     \
        int rc_ = (expr);    \
        if (rc_) return rc_; \
    } while (0)

// one problem after validation: everything the device passes need
struct Prepared {
    int A = 0, t = 0, l = 0, k = 0, s = 0, m = 0;
    int n_min = 0, n_max = 0;
    int64_t n_total = 0, x = 0;
    std::vector<uint8_t> ascii;
    std::vector<int64_t> off;
    std::vector<uint32_t> masks;
    std::vector<double> bg;
};

int prepare(const pm_problem &P, int index, Prepared &Q)
{
    const int A = P.alphabet;
    if (A != 4 && A != 20) return fail(PM_EINVAL, "problem %d: alphabet must be 4 or 20", index);
    if (P.t < 1 || !P.seqs || !P.n) return fail(PM_EINVAL, "problem %d: need t >= 1 sequences", index);
    const int l = P.l;
    int64_t n_total = 0;
    int n_min = 0x7fffffff, n_max = 0;
    for (int i = 0; i < P.t; ++i) {
        if (!P.seqs[i] || P.n[i] < 0)
            return fail(PM_EINVAL, "problem %d: sequence %d is NULL or has negative length", index, i);
        n_total += P.n[i];
        n_min = std::min(n_min, (int)P.n[i]);
        n_max = std::max(n_max, (int)P.n[i]);
    }
    if (l < 1 || l > 32 || n_min < l) return fail(PM_EINVAL, "problem %d: need 1 <= l <= 32 and l <= every n_i", index);
    if (n_total >= (1ll << 31)) return fail(PM_ERANGE, "problem %d: n_total must stay below 2^31", index);
    const int64_t x = n_total - (int64_t)P.t * (l - 1);
    int k = P.k, s = P.s, m = P.m;
    if (P.masks && P.m < 1) return fail(PM_EINVAL, "problem %d: masks given, so m must count them (m >= 1)", index);
    if (k <= 0 || s <= 0 || m <= 0) {
        int ak, as, am;
        PM_CALL(pm_auto_params(A, P.t, x, l, P.d, 0.95, &ak, &as, &am));
        if (k <= 0) k = ak;
        if (s <= 0) s = as;
        if (m <= 0) m = am;
    }
    if (k < 1 || k > l) return fail(PM_EINVAL, "problem %d: need 1 <= k <= l", index);
    Q.A = A;
    Q.t = P.t;
    Q.l = l;
    Q.k = k;
    Q.s = s;
    Q.m = m;
    Q.n_min = n_min;
    Q.n_max = n_max;
    Q.n_total = n_total;
    Q.x = x;
    Q.ascii.resize((size_t)n_total);
    Q.off.assign(P.t + 1, 0);
    for (int i = 0; i < P.t; ++i) {
        memcpy(Q.ascii.data() + Q.off[i], P.seqs[i], (size_t)P.n[i]);
        Q.off[i + 1] = Q.off[i] + P.n[i];
    }
    Q.masks.resize((size_t)m);
    if (P.masks) memcpy(Q.masks.data(), P.masks, sizeof(uint32_t) * m);
    else PM_CALL(pm_masks_from_seed(P.seed, l, k, m, Q.masks.data()));
    for (int j = 0; j < m; ++j)
        if (__builtin_popcount(Q.masks[j]) != k || (l < 32 && (Q.masks[j] >> l)))
            return fail(PM_EINVAL, "problem %d: mask %d does not keep exactly k=%d of l=%d positions", index, j, k, l);
    Q.bg.assign(A, 0.0);
    const char *letters = A == 4 ? "ACTG" : "ARNDCQEGHILKMFPSTWYV";
    if (P.bg) {
        double tot = 0;
        for (int c = 0; c < A; ++c) {
            if (!(P.bg[c] > 0)) return fail(PM_EINVAL, "problem %d: background frequencies must be positive", index);
            tot += P.bg[c];
        }
        for (int c = 0; c < A; ++c) Q.bg[c] = P.bg[c] / tot;
    } else {
        // composition of the input (the background is fixed, never re-estimated)
        std::vector<double> cnt(A, 0.0);
        for (int64_t g = 0; g < n_total; ++g) {
            const char ch = (char)Q.ascii[g];
            const char u = (ch >= 'a' && ch <= 'z') ? (char)(ch - 'a' + 'A') : ch;
            const char *f = u ? strchr(letters, u) : nullptr;
            if (!f) return fail(PM_EINVAL, "problem %d: a sequence holds a symbol outside the alphabet", index);
            cnt[f - letters] += 1;
        }
        for (int c = 0; c < A; ++c) Q.bg[c] = cnt[c] / (double)n_total;
        for (int c = 0; c < A; ++c)
            if (!(Q.bg[c] > 0))
                return fail(PM_EINVAL, "problem %d: letter %c never occurs; pass a background", index, letters[c]);
    }
    return PM_OK;
}

void empty_result(pm_result &R, const Prepared &Q)
{
    R.k = Q.k;
    R.s = Q.s;
    R.m = Q.m;
    R.n_enriched = 0;
    R.n_refined = 0;
    R.fallback_used = 0;
    R.best_trial = -1;
    R.best_key = 0;
    R.J = R.llr = -INFINITY;
    if (R.consensus) R.consensus[0] = 0;
}

// ---------------------------------------------------------------- one problem
int run_single(const Prepared &Q, const pm_options &O, pm_result &R, hipStream_t st)
{
    const int A = Q.A, l = Q.l, k = Q.k, s = Q.s, m = Q.m, t = Q.t;
    const int64_t n_total = Q.n_total;
    empty_result(R, Q);
    const int64_t nw = pm_packed_words(A, n_total);
    DevBuf d_ascii, d_off, d_packed, d_masks, d_status, d_nout, d_ws;
    PM_CALL(d_ascii.alloc(n_total));
    PM_CALL(d_off.alloc(sizeof(int64_t) * (t + 1)));
    PM_CALL(d_packed.alloc(sizeof(uint32_t) * nw));
    PM_CALL(d_masks.alloc(sizeof(uint32_t) * m));
    PM_CALL(d_status.alloc(sizeof(uint32_t)));
    PM_CALL(d_nout.alloc(sizeof(int64_t) * 2));
    PM_TRY(hipMemcpyAsync(d_ascii.p, Q.ascii.data(), n_total, hipMemcpyHostToDevice, st));
    PM_TRY(hipMemcpyAsync(d_off.p, Q.off.data(), sizeof(int64_t) * (t + 1), hipMemcpyHostToDevice, st));
    PM_TRY(hipMemcpyAsync(d_masks.p, Q.masks.data(), sizeof(uint32_t) * m, hipMemcpyHostToDevice, st));
    PM_TRY(hipMemsetAsync(d_status.p, 0, sizeof(uint32_t), st));

    pm_seqs S{A, t, n_total, Q.n_min, Q.n_max, d_off.as<int64_t>(), d_packed.as<uint32_t>()};
    PM_CALL(pm_pack(A, d_ascii.as<uint8_t>(), n_total, d_packed.as<uint32_t>(), d_status.as<uint32_t>(), st));
    // the fused selection (keys and counts stay on chip; large key spaces are
    // sorted instead of counted): a sizing pass with empty capacities, then
    // the lists
    const size_t hws = pm_hash_select_workspace(&S, l, k, m);
    if (!hws) return fail(PM_ERANGE, "k=%d is beyond the selection's range for this alphabet", k);
    PM_CALL(d_ws.alloc(hws));
    PM_CALL(bucket_hash_select(&S, l, k, d_masks.as<uint32_t>(), m, (uint32_t)s, nullptr, 0, nullptr, 0,
                               d_nout.as<int64_t>(), d_ws.p, hws, nullptr, st));
    int64_t nout[2];
    uint32_t status = 0;
    PM_TRY(hipMemcpyAsync(nout, d_nout.p, sizeof(nout), hipMemcpyDeviceToHost, st));
    PM_TRY(hipMemcpyAsync(&status, d_status.p, sizeof(status), hipMemcpyDeviceToHost, st));
    PM_TRY(hipStreamSynchronize(st));
    if (status & PM_STATUS_BAD_SYMBOL) return fail(PM_EINVAL, "a sequence holds a symbol outside the alphabet");
    const int64_t nbk = nout[0], nmem = nout[1];
    R.n_enriched = nbk;
    if (nbk == 0) return PM_OK;
    DevBuf d_bk, d_mem, d_prof, d_bg, d_th0, d_th, d_J, d_llr, d_sites, d_best, d_cons, d_emws;
    PM_CALL(d_bk.alloc(sizeof(pm_bucket) * nbk));
    PM_CALL(d_mem.alloc(sizeof(uint32_t) * nmem));
    PM_CALL(bucket_hash_select(&S, l, k, d_masks.as<uint32_t>(), m, (uint32_t)s, d_bk.as<pm_bucket>(), nbk,
                               d_mem.as<uint32_t>(), nmem, d_nout.as<int64_t>(), d_ws.p, hws,
                               d_status.as<uint32_t>(), st));
    d_ws.release();

    const int AL = A * l;
    const int it1 = O.em_iters + 1;
    PM_CALL(d_prof.alloc(sizeof(uint32_t) * nbk * AL));
    PM_CALL(d_bg.alloc(sizeof(double) * A));
    PM_CALL(d_th0.alloc(sizeof(double) * nbk * AL));
    PM_CALL(d_th.alloc(sizeof(double) * nbk * AL));
    PM_CALL(d_J.alloc(sizeof(double) * nbk * it1));
    PM_CALL(d_llr.alloc(sizeof(double) * nbk * it1));
    PM_CALL(d_sites.alloc(sizeof(int32_t) * nbk * t));
    PM_CALL(d_best.alloc(sizeof(int64_t)));
    PM_CALL(d_cons.alloc(l + 1));
    const size_t em_ws = pm_em_workspace(&S, l, O.precision);
    if (em_ws) PM_CALL(d_emws.alloc(em_ws));
    PM_TRY(hipMemcpyAsync(d_bg.p, Q.bg.data(), sizeof(double) * A, hipMemcpyHostToDevice, st));
    PM_CALL(bucket_profile(&S, l, d_bk.as<pm_bucket>(), d_mem.as<uint32_t>(), nmem, nbk, nullptr,
                           d_prof.as<uint32_t>(), st));
    PM_CALL(theta_init(A, l, d_prof.as<uint32_t>(), nbk, nullptr, d_bg.as<double>(), O.beta, d_th0.as<double>(), st));
    PM_CALL(em_refine(&S, l, d_th0.as<double>(), d_bg.as<double>(), nbk, nullptr, O.em_iters, O.beta, O.precision,
                      d_th.as<double>(), d_J.as<double>(), d_llr.as<double>(), d_sites.as<int32_t>(), d_emws.p, em_ws,
                      st));
    PM_CALL(em_best(d_J.as<double>(), nbk, nullptr, O.em_iters, d_th.as<double>(), A, l, d_best.as<int64_t>(),
                    d_cons.as<char>(), st));
    R.n_refined = nbk;
    int64_t best = -1;
    PM_TRY(hipMemcpyAsync(&best, d_best.p, sizeof(best), hipMemcpyDeviceToHost, st));
    PM_TRY(hipStreamSynchronize(st));
    if (best < 0) return PM_OK;
    pm_bucket bk;
    PM_TRY(hipMemcpyAsync(&bk, d_bk.as<pm_bucket>() + best, sizeof(bk), hipMemcpyDeviceToHost, st));
    PM_TRY(hipMemcpyAsync(&R.J, d_J.as<double>() + best * it1 + O.em_iters, sizeof(double), hipMemcpyDeviceToHost, st));
    PM_TRY(hipMemcpyAsync(&R.llr, d_llr.as<double>() + best * it1 + O.em_iters, sizeof(double), hipMemcpyDeviceToHost,
                          st));
    if (R.consensus) PM_TRY(hipMemcpyAsync(R.consensus, d_cons.p, l + 1, hipMemcpyDeviceToHost, st));
    if (R.sites)
        PM_TRY(hipMemcpyAsync(R.sites, d_sites.as<int32_t>() + best * t, sizeof(int32_t) * t, hipMemcpyDeviceToHost,
                              st));
    if (R.theta)
        PM_TRY(hipMemcpyAsync(R.theta, d_th.as<double>() + best * AL, sizeof(double) * AL, hipMemcpyDeviceToHost, st));
    PM_TRY(hipStreamSynchronize(st));
    R.best_trial = (int32_t)bk.trial;
    R.best_key = bk.key;
    return PM_OK;
}

// ---------------------------------------------------------------- triage weights
struct TriageModel {
    std::vector<float> params, mu, sd;
    double pooled = 0;
    std::map<int, double> by_l;
    double threshold(int l) const
    {
        auto it = by_l.find(l);
        return it == by_l.end() ? pooled : it->second;
    }
};

int read_triage(const char *path, TriageModel &T)
{
    if (!path) return fail(PM_EINVAL, "triage needs a weights file (triage_weights is NULL)");
    FILE *f = fopen(path, "rb");
    if (!f) return fail(PM_EINVAL, "cannot open triage weights %s", path);
    auto rd = [&](void *dst, size_t n) { return fread(dst, 1, n, f) == n; };
    char magic[8];
    int32_t np = 0, ni = 0, nl = 0;
    bool ok = rd(magic, 8) && memcmp(magic, "PMTRIAG1", 8) == 0 && rd(&np, 4) && rd(&ni, 4) &&
              np == PM_TRIAGE_PARAMS && ni == PM_TRIAGE_INPUTS;
    if (ok) {
        T.params.resize(np);
        T.mu.resize(ni);
        T.sd.resize(ni);
        ok = rd(T.params.data(), 4 * (size_t)np) && rd(T.mu.data(), 4 * (size_t)ni) && rd(T.sd.data(), 4 * (size_t)ni) &&
             rd(&T.pooled, 8) && rd(&nl, 4) && nl >= 0 && nl <= 64;
    }
    for (int q = 0; ok && q < nl; ++q) {
        int32_t l = 0;
        double v = 0;
        ok = rd(&l, 4) && rd(&v, 8);
        if (ok) T.by_l[l] = v;
    }
    fclose(f);
    if (!ok) return fail(PM_EINVAL, "%s is not a triage weights file (PMTRIAG1, %d parameters)", path, PM_TRIAGE_PARAMS);
    return PM_OK;
}

// ---------------------------------------------------------------- gather
// Per instance, the answer's objective, log-likelihood ratio, model, sites and
// bucket, from the list whose winner is the final one: list 1 when its best
// (mapped through index1 when given) is the final pick, else list 2.
struct GatherList {
    const int64_t *best;   // [P] index into the list, or -1
    const int64_t *index;  // [n] original bucket index of each list entry, or NULL (identity)
    const double *J, *llr, *theta;
    const int32_t *sites;
    const pm_bucket *buckets;
};

__global__ void k_gather_best(int P, const int64_t *final_best, GatherList L1, GatherList L2, int it1, int t_max,
                              int AL, int32_t *which, double *J, double *llr, double *theta, int32_t *sites,
                              pm_bucket *bk)
{
    const int p = blockIdx.x;
    if (p >= P) return;
    const int64_t fb = final_best ? final_best[p] : L1.best[p];
    int src = 0;
    int64_t i = -1;
    if (fb >= 0) {
        const int64_t b1 = L1.best[p];
        if (b1 >= 0 && (L1.index ? L1.index[b1] : b1) == fb) {
            src = 1;
            i = b1;
        } else if (L2.best && L2.best[p] >= 0) {
            src = 2;
            i = L2.best[p];
        }
    }
    if (threadIdx.x == 0) which[p] = src;
    if (src == 0) return;
    const GatherList L = src == 1 ? L1 : L2;
    if (threadIdx.x == 0) {
        J[p] = L.J[i * it1 + it1 - 1];
        llr[p] = L.llr[i * it1 + it1 - 1];
        bk[p] = L.buckets[i];
    }
    for (int q = threadIdx.x; q < AL; q += blockDim.x) theta[(int64_t)p * AL + q] = L.theta[i * AL + q];
    for (int q = threadIdx.x; q < t_max; q += blockDim.x) sites[(int64_t)p * t_max + q] = L.sites[i * t_max + q];
}

// entries of a bucket list per instance (buckets' trial fields are items)
__global__ void k_count_by_instance(const pm_bucket *bk, const int64_t *n_dev, int64_t cap, const int32_t *item_inst,
                                    unsigned long long *cnt)
{
    int64_t n = n_dev ? *n_dev : cap;
    if (n > cap) n = cap;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < n; b += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(cnt + item_inst[bk[b].trial], 1ull);
}

// ---------------------------------------------------------------- a batch of problems
// Device inputs of one group of problems, packed once: every instance's words,
// offsets and masks, and the instance table over the whole group.
struct GroupDev {
    int A, l, k, s, t_max;
    DevBuf packed, off, masks, bg, status;
    std::vector<pm_inst> inst;     // host table over the group (device pointers set)
    std::vector<int64_t> nb, nm;   // enriched buckets and members of every instance
};

// Bytes one enriched bucket costs through the rest of the path (lists,
// profiles, models, objectives, sites; the two triage lists when on).
size_t bytes_per_bucket(int AL, int it1, int t_max, bool triage)
{
    size_t b = sizeof(pm_bucket) + (size_t)AL * (4 + 8 + 8) + (size_t)it1 * 16 + (size_t)t_max * 4;
    if (triage)
        b += (size_t)PM_TRIAGE_INPUTS * 4 + 4 + 1 +
             2 * (sizeof(pm_bucket) + (size_t)AL * 16 + 8 + (size_t)it1 * 16 + (size_t)t_max * 4);
    return b;
}

// The sub-batch of instances [p0, p1): its own instance table (items and key
// bases restarting at 0), the fused selection, profiles, theta^0, EM (all
// buckets, or triaged), the best model of every instance, copied into Rs.
int run_sub(GroupDev &D, int p0, int p1, const std::vector<const Prepared *> &G, const std::vector<pm_result *> &Rs,
            const pm_options &O, const TriageModel *tri, hipStream_t st)
{
    const int A = D.A, l = D.l, k = D.k, s = D.s, P = p1 - p0, t_max = D.t_max;
    const int iters = O.em_iters, it1 = iters + 1, AL = A * l;
    std::vector<pm_inst> inst(D.inst.begin() + p0, D.inst.begin() + p1);
    const int64_t item0 = inst[0].first_item;
    int64_t items = 0, key = 0;
    for (pm_inst &I : inst) {
        I.first_item = (int32_t)items;
        I.key_base = key;
        items += I.m;
        key += (int64_t)I.m * I.x;
    }
    std::vector<int32_t> item_inst((size_t)items);
    for (int p = 0; p < P; ++p)
        for (int j = 0; j < inst[p].m; ++j) item_inst[inst[p].first_item + j] = p;
    DevBuf d_inst, d_item, d_nout, d_ws;
    PM_CALL(d_inst.alloc(sizeof(pm_inst) * P));
    PM_CALL(d_item.alloc(sizeof(int32_t) * items));
    PM_CALL(d_nout.alloc(sizeof(int64_t) * 2));
    PM_TRY(hipMemcpyAsync(d_inst.p, inst.data(), sizeof(pm_inst) * P, hipMemcpyHostToDevice, st));
    PM_TRY(hipMemcpyAsync(d_item.p, item_inst.data(), sizeof(int32_t) * items, hipMemcpyHostToDevice, st));
    const pm_batch Bt{A, l, k, P, (int32_t)items, d_inst.as<pm_inst>(), inst.data(), d_item.as<int32_t>()};
    const uint32_t *masks = D.masks.as<uint32_t>() + item0;
    int64_t nbk = 0, nmem = 0;
    for (int p = p0; p < p1; ++p) {
        nbk += D.nb[p];
        nmem += D.nm[p];
    }
    if (nbk == 0) return PM_OK;
    const size_t hws = pm_hash_select_batch_workspace(&Bt);
    if (!hws) return PM_ERANGE;
    DevBuf d_bk, d_mem, d_prof, d_th0, d_th, d_J, d_llr, d_sites, d_best, d_cons, d_emws;
    PM_CALL(d_ws.alloc(hws));
    PM_CALL(d_bk.alloc(sizeof(pm_bucket) * nbk));
    PM_CALL(d_mem.alloc(sizeof(uint32_t) * nmem));
    PM_CALL(bucket_hash_select_batch(&Bt, masks, (uint32_t)s, d_bk.as<pm_bucket>(), nbk, d_mem.as<uint32_t>(), nmem,
                                     d_nout.as<int64_t>(), d_ws.p, hws, D.status.as<uint32_t>(), st));
    d_ws.release();
    PM_CALL(d_prof.alloc(sizeof(uint32_t) * nbk * AL));
    PM_CALL(d_th0.alloc(sizeof(double) * nbk * AL));
    PM_CALL(d_best.alloc(sizeof(int64_t) * P));
    PM_CALL(d_cons.alloc((size_t)P * (l + 1)));
    PM_CALL(bucket_profile_batch(&Bt, d_bk.as<pm_bucket>(), d_mem.as<uint32_t>(), nmem, nbk, nullptr,
                                 d_prof.as<uint32_t>(), st));
    d_mem.release();
    PM_CALL(theta_init(A, l, d_prof.as<uint32_t>(), nbk, nullptr, D.bg.as<double>(), O.beta, d_th0.as<double>(), st));
    const size_t em_ws = pm_em_batch_workspace(&Bt, O.precision);
    if (em_ws) PM_CALL(d_emws.alloc(em_ws));

    // per-instance outputs gathered on the device
    DevBuf g_which, g_J, g_llr, g_theta, g_sites, g_bk, d_cnt;
    PM_CALL(g_which.alloc(sizeof(int32_t) * P));
    PM_CALL(g_J.alloc(sizeof(double) * P));
    PM_CALL(g_llr.alloc(sizeof(double) * P));
    PM_CALL(g_theta.alloc(sizeof(double) * P * AL));
    PM_CALL(g_sites.alloc(sizeof(int32_t) * P * t_max));
    PM_CALL(g_bk.alloc(sizeof(pm_bucket) * P));
    std::vector<int32_t> fell(P, 0);
    std::vector<unsigned long long> refined(P, 0);

    if (!tri) {
        d_prof.release();
        PM_CALL(d_th.alloc(sizeof(double) * nbk * AL));
        PM_CALL(d_J.alloc(sizeof(double) * nbk * it1));
        PM_CALL(d_llr.alloc(sizeof(double) * nbk * it1));
        PM_CALL(d_sites.alloc(sizeof(int32_t) * nbk * t_max));
        PM_CALL(em_refine_batch(&Bt, d_bk.as<pm_bucket>(), d_th0.as<double>(), D.bg.as<double>(), nbk, nullptr, iters,
                                O.beta, O.precision, d_th.as<double>(), d_J.as<double>(), d_llr.as<double>(),
                                d_sites.as<int32_t>(), d_emws.p, em_ws, st));
        PM_CALL(em_best_batch(&Bt, d_bk.as<pm_bucket>(), d_J.as<double>(), nbk, nullptr, iters, d_th.as<double>(),
                              d_best.as<int64_t>(), d_cons.as<char>(), st));
        const GatherList L1{d_best.as<int64_t>(), nullptr, d_J.as<double>(), d_llr.as<double>(), d_th.as<double>(),
                            d_sites.as<int32_t>(), d_bk.as<pm_bucket>()};
        const GatherList L2{};
        hipLaunchKernelGGL(k_gather_best, dim3(P), dim3(64), 0, st, P, nullptr, L1, L2, it1, t_max, AL,
                           g_which.as<int32_t>(), g_J.as<double>(), g_llr.as<double>(), g_theta.as<double>(),
                           g_sites.as<int32_t>(), g_bk.as<pm_bucket>());
        PM_LAUNCHED();
        for (int p = 0; p < P; ++p) refined[p] = (unsigned long long)D.nb[p0 + p];
    } else {
        // scores of every bucket, then the two refinement lists
        DevBuf t_params, t_mu, t_sd, t_packed, t_feat, t_score, t_taken, t_sws, t_fell, t_z;
        PM_CALL(t_params.alloc(sizeof(float) * tri->params.size()));
        PM_CALL(t_mu.alloc(sizeof(float) * PM_TRIAGE_INPUTS));
        PM_CALL(t_sd.alloc(sizeof(float) * PM_TRIAGE_INPUTS));
        PM_CALL(t_packed.alloc(pm_triage_packed_bytes()));
        PM_CALL(t_feat.alloc(sizeof(float) * nbk * PM_TRIAGE_INPUTS));
        PM_CALL(t_score.alloc(sizeof(float) * nbk));
        PM_CALL(t_taken.alloc(nbk));
        const size_t sws = pm_triage_select_workspace(P, nbk);
        PM_CALL(t_sws.alloc(sws));
        PM_CALL(t_fell.alloc(sizeof(int32_t) * P));
        PM_CALL(t_z.alloc(sizeof(double) * P));
        PM_TRY(hipMemcpyAsync(t_params.p, tri->params.data(), sizeof(float) * tri->params.size(), hipMemcpyHostToDevice,
                              st));
        PM_TRY(hipMemcpyAsync(t_mu.p, tri->mu.data(), sizeof(float) * PM_TRIAGE_INPUTS, hipMemcpyHostToDevice, st));
        PM_TRY(hipMemcpyAsync(t_sd.p, tri->sd.data(), sizeof(float) * PM_TRIAGE_INPUTS, hipMemcpyHostToDevice, st));
        PM_CALL(triage_pack(t_params.as<float>(), t_packed.p, st));
        PM_CALL(triage_features(l, d_prof.as<uint32_t>(), nbk, nullptr, D.bg.as<double>(), t_mu.as<float>(),
                                t_sd.as<float>(), t_feat.as<float>(), st));
        PM_CALL(triage_forward(t_packed.p, t_feat.as<float>(), nbk, nullptr, t_score.as<float>(), st));
        d_prof.release();
        t_feat.release();
        struct List {
            DevBuf bk, th0, index, n, th, J, llr, sites, best;
        } L[2];
        for (auto &X : L) {
            PM_CALL(X.bk.alloc(sizeof(pm_bucket) * nbk));
            PM_CALL(X.th0.alloc(sizeof(double) * nbk * AL));
            PM_CALL(X.index.alloc(sizeof(int64_t) * nbk));
            PM_CALL(X.n.alloc(sizeof(int64_t)));
            PM_CALL(X.th.alloc(sizeof(double) * nbk * AL));
            PM_CALL(X.J.alloc(sizeof(double) * nbk * it1));
            PM_CALL(X.llr.alloc(sizeof(double) * nbk * it1));
            PM_CALL(X.sites.alloc(sizeof(int32_t) * nbk * t_max));
            PM_CALL(X.best.alloc(sizeof(int64_t) * P));
        }
        auto refine = [&](List &X) -> int {
            PM_CALL(em_refine_batch(&Bt, X.bk.as<pm_bucket>(), X.th0.as<double>(), D.bg.as<double>(), nbk,
                                    X.n.as<int64_t>(), iters, O.beta, O.precision, X.th.as<double>(), X.J.as<double>(),
                                    X.llr.as<double>(), X.sites.as<int32_t>(), d_emws.p, em_ws, st));
            return em_best_batch(&Bt, X.bk.as<pm_bucket>(), X.J.as<double>(), nbk, X.n.as<int64_t>(), iters,
                                 X.th.as<double>(), X.best.as<int64_t>(), nullptr, st);
        };
        PM_CALL(triage_select(&Bt, d_bk.as<pm_bucket>(), t_score.as<float>(), nbk, nullptr, O.triage_frac,
                              d_th0.as<double>(), A, l, t_taken.as<uint8_t>(), L[0].bk.as<pm_bucket>(),
                              L[0].th0.as<double>(), L[0].index.as<int64_t>(), L[0].n.as<int64_t>(), t_sws.p, sws, st));
        PM_CALL(refine(L[0]));
        PM_CALL(triage_fallback_select(&Bt, d_bk.as<pm_bucket>(), nbk, nullptr, L[0].bk.as<pm_bucket>(),
                                       L[0].n.as<int64_t>(), L[0].best.as<int64_t>(), L[0].J.as<double>(), iters,
                                       tri->threshold(l), d_th0.as<double>(), A, l, t_taken.as<uint8_t>(),
                                       L[1].bk.as<pm_bucket>(), L[1].th0.as<double>(), L[1].index.as<int64_t>(),
                                       L[1].n.as<int64_t>(), t_fell.as<int32_t>(), t_z.as<double>(), t_sws.p, sws, st));
        PM_CALL(refine(L[1]));
        PM_CALL(triage_merge_best(P, A, l, iters, L[0].best.as<int64_t>(), L[0].index.as<int64_t>(),
                                  L[0].J.as<double>(), L[0].th.as<double>(), L[1].best.as<int64_t>(),
                                  L[1].index.as<int64_t>(), L[1].J.as<double>(), L[1].th.as<double>(),
                                  d_best.as<int64_t>(), d_cons.as<char>(), st));
        const GatherList G1{L[0].best.as<int64_t>(), L[0].index.as<int64_t>(), L[0].J.as<double>(),
                            L[0].llr.as<double>(), L[0].th.as<double>(), L[0].sites.as<int32_t>(),
                            L[0].bk.as<pm_bucket>()};
        const GatherList G2{L[1].best.as<int64_t>(), L[1].index.as<int64_t>(), L[1].J.as<double>(),
                            L[1].llr.as<double>(), L[1].th.as<double>(), L[1].sites.as<int32_t>(),
                            L[1].bk.as<pm_bucket>()};
        hipLaunchKernelGGL(k_gather_best, dim3(P), dim3(64), 0, st, P, d_best.as<int64_t>(), G1, G2, it1, t_max, AL,
                           g_which.as<int32_t>(), g_J.as<double>(), g_llr.as<double>(), g_theta.as<double>(),
                           g_sites.as<int32_t>(), g_bk.as<pm_bucket>());
        PM_LAUNCHED();
        PM_CALL(d_cnt.alloc(sizeof(unsigned long long) * P));
        PM_TRY(hipMemsetAsync(d_cnt.p, 0, sizeof(unsigned long long) * P, st));
        for (auto &X : L) {
            hipLaunchKernelGGL(k_count_by_instance, dim3(1024), dim3(256), 0, st, X.bk.as<pm_bucket>(),
                               X.n.as<int64_t>(), nbk, d_item.as<int32_t>(), d_cnt.as<unsigned long long>());
            PM_LAUNCHED();
        }
        PM_TRY(hipMemcpyAsync(refined.data(), d_cnt.p, sizeof(unsigned long long) * P, hipMemcpyDeviceToHost, st));
        PM_TRY(hipMemcpyAsync(fell.data(), t_fell.p, sizeof(int32_t) * P, hipMemcpyDeviceToHost, st));
        PM_TRY(hipStreamSynchronize(st));  // the lists are freed at the end of this scope
    }

    std::vector<int32_t> which(P);
    std::vector<double> J(P), llr(P), theta((size_t)P * AL);
    std::vector<int32_t> sites((size_t)P * t_max);
    std::vector<pm_bucket> bk(P);
    std::vector<char> cons((size_t)P * (l + 1));
    uint32_t status = 0;
    PM_TRY(hipMemcpyAsync(which.data(), g_which.p, sizeof(int32_t) * P, hipMemcpyDeviceToHost, st));
    PM_TRY(hipMemcpyAsync(J.data(), g_J.p, sizeof(double) * P, hipMemcpyDeviceToHost, st));
    PM_TRY(hipMemcpyAsync(llr.data(), g_llr.p, sizeof(double) * P, hipMemcpyDeviceToHost, st));
    PM_TRY(hipMemcpyAsync(theta.data(), g_theta.p, sizeof(double) * P * AL, hipMemcpyDeviceToHost, st));
    PM_TRY(hipMemcpyAsync(sites.data(), g_sites.p, sizeof(int32_t) * P * t_max, hipMemcpyDeviceToHost, st));
    PM_TRY(hipMemcpyAsync(bk.data(), g_bk.p, sizeof(pm_bucket) * P, hipMemcpyDeviceToHost, st));
    PM_TRY(hipMemcpyAsync(cons.data(), d_cons.p, (size_t)P * (l + 1), hipMemcpyDeviceToHost, st));
    PM_TRY(hipMemcpyAsync(&status, D.status.p, sizeof(status), hipMemcpyDeviceToHost, st));
    PM_TRY(hipStreamSynchronize(st));
    if (status & PM_STATUS_CAPACITY) return fail(PM_EDEVICE, "bucket lists overflowed their counted sizes");
    for (int p = 0; p < P; ++p) {
        pm_result &R = *Rs[p0 + p];
        R.n_refined = (int64_t)refined[p];
        R.fallback_used = fell[p];
        if (which[p] == 0) continue;
        R.J = J[p];
        R.llr = llr[p];
        R.best_trial = (int32_t)bk[p].trial - inst[p].first_item;
        R.best_key = bk[p].key;
        if (R.consensus) memcpy(R.consensus, cons.data() + (size_t)p * (l + 1), l + 1);
        if (R.sites) memcpy(R.sites, sites.data() + (size_t)p * t_max, sizeof(int32_t) * G[p0 + p]->t);
        if (R.theta) memcpy(R.theta, theta.data() + (size_t)p * AL, sizeof(double) * AL);
    }
    return PM_OK;
}

// A group of problems sharing alphabet, l, k, s and background: packed once,
// counted once over all its trials (fused selection, counting pass only),
// then streamed through the rest of the path in sub-batches of whole
// instances whose buckets fit the memory budget.
int run_group(const std::vector<const Prepared *> &G, const std::vector<pm_result *> &Rs, const pm_options &O,
              const TriageModel *tri, hipStream_t st)
{
    const Prepared &q0 = *G[0];
    const int A = q0.A, l = q0.l, k = q0.k, s = q0.s, P = (int)G.size();
    const int per = A == 4 ? 16 : 6;
    const int AL = A * l;
    for (int p = 0; p < P; ++p) empty_result(*Rs[p], *G[p]);

    // host layout: instance p's ASCII padded with code-0 letters to whole
    // packed words (including pm_pack's four padding words), its local offsets
    std::vector<int64_t> word_base(P), off_base(P);
    int64_t words = 0, offs = 0, items = 0;
    int t_max = 0;
    for (int p = 0; p < P; ++p) {
        word_base[p] = words;
        off_base[p] = offs;
        words += pm_packed_words(A, G[p]->n_total);
        offs += G[p]->t + 1;
        items += G[p]->m;
        t_max = std::max(t_max, G[p]->t);
    }
    if (items > 0x7fffffff) return fail(PM_ERANGE, "more than 2^31 - 1 trials in one batch");
    std::vector<uint8_t> ascii((size_t)(words * per), (uint8_t)'A');
    std::vector<int64_t> off((size_t)offs);
    std::vector<uint32_t> masks((size_t)items);
    std::vector<int32_t> item_inst((size_t)items);
    GroupDev D;
    D.A = A;
    D.l = l;
    D.k = k;
    D.s = s;
    D.t_max = t_max;
    D.inst.resize(P);
    {
        int64_t it = 0, key = 0;
        for (int p = 0; p < P; ++p) {
            const Prepared &Q = *G[p];
            memcpy(ascii.data() + word_base[p] * per, Q.ascii.data(), (size_t)Q.n_total);
            memcpy(off.data() + off_base[p], Q.off.data(), sizeof(int64_t) * (Q.t + 1));
            memcpy(masks.data() + it, Q.masks.data(), sizeof(uint32_t) * Q.m);
            for (int j = 0; j < Q.m; ++j) item_inst[it + j] = p;
            pm_inst &I = D.inst[p];
            I.n_total = Q.n_total;
            I.x = Q.x;
            I.key_base = key;
            I.t = Q.t;
            I.n_min = Q.n_min;
            I.m = Q.m;
            I.first_item = (int32_t)it;
            it += Q.m;
            key += (int64_t)Q.m * Q.x;
        }
    }
    DevBuf d_ascii, d_inst, d_item, d_nout, d_ws;
    PM_CALL(d_ascii.alloc(ascii.size()));
    PM_CALL(D.off.alloc(sizeof(int64_t) * off.size()));
    PM_CALL(D.packed.alloc(sizeof(uint32_t) * pm_packed_words(A, (int64_t)ascii.size())));
    PM_CALL(D.masks.alloc(sizeof(uint32_t) * items));
    PM_CALL(D.bg.alloc(sizeof(double) * A));
    PM_CALL(D.status.alloc(sizeof(uint32_t)));
    PM_CALL(d_inst.alloc(sizeof(pm_inst) * P));
    PM_CALL(d_item.alloc(sizeof(int32_t) * items));
    PM_CALL(d_nout.alloc(sizeof(int64_t) * 2));
    for (int p = 0; p < P; ++p) {
        D.inst[p].offsets = D.off.as<int64_t>() + off_base[p];
        D.inst[p].packed = D.packed.as<uint32_t>() + word_base[p];
    }
    PM_TRY(hipMemcpyAsync(d_ascii.p, ascii.data(), ascii.size(), hipMemcpyHostToDevice, st));
    PM_TRY(hipMemcpyAsync(D.off.p, off.data(), sizeof(int64_t) * off.size(), hipMemcpyHostToDevice, st));
    PM_TRY(hipMemcpyAsync(D.masks.p, masks.data(), sizeof(uint32_t) * items, hipMemcpyHostToDevice, st));
    PM_TRY(hipMemcpyAsync(d_inst.p, D.inst.data(), sizeof(pm_inst) * P, hipMemcpyHostToDevice, st));
    PM_TRY(hipMemcpyAsync(d_item.p, item_inst.data(), sizeof(int32_t) * items, hipMemcpyHostToDevice, st));
    PM_TRY(hipMemcpyAsync(D.bg.p, q0.bg.data(), sizeof(double) * A, hipMemcpyHostToDevice, st));
    PM_TRY(hipMemsetAsync(D.status.p, 0, sizeof(uint32_t), st));
    PM_CALL(pm_pack(A, d_ascii.as<uint8_t>(), (int64_t)ascii.size(), D.packed.as<uint32_t>(), D.status.as<uint32_t>(),
                    st));
    const pm_batch Bt{A, l, k, P, (int32_t)items, d_inst.as<pm_inst>(), D.inst.data(), d_item.as<int32_t>()};
    // counting pass over every trial: totals per (item, key-range slice)
    const size_t hws = pm_hash_select_batch_workspace(&Bt);
    if (!hws) return PM_ERANGE;
    PM_CALL(d_ws.alloc(hws));
    PM_CALL(bucket_hash_select_batch(&Bt, D.masks.as<uint32_t>(), (uint32_t)s, nullptr, 0, nullptr, 0,
                                     d_nout.as<int64_t>(), d_ws.p, hws, nullptr, st));
    const int64_t entries = (int64_t)((hws - 256) / (4 * sizeof(int64_t)));
    const int64_t nslices = entries / items;
    std::vector<int64_t> tot((size_t)(2 * entries));
    uint32_t status = 0;
    PM_TRY(hipMemcpyAsync(tot.data(), d_ws.p, sizeof(int64_t) * 2 * entries, hipMemcpyDeviceToHost, st));
    PM_TRY(hipMemcpyAsync(&status, D.status.p, sizeof(status), hipMemcpyDeviceToHost, st));
    PM_TRY(hipStreamSynchronize(st));
    d_ws.release();
    if (status & PM_STATUS_BAD_SYMBOL) return fail(PM_EINVAL, "a sequence holds a symbol outside the alphabet");
    D.nb.assign(P, 0);
    D.nm.assign(P, 0);
    for (int p = 0; p < P; ++p) {
        const int64_t e0 = (int64_t)D.inst[p].first_item * nslices, e1 = e0 + (int64_t)D.inst[p].m * nslices;
        for (int64_t e = e0; e < e1; ++e) {
            D.nb[p] += tot[e];
            D.nm[p] += tot[entries + e];
        }
        Rs[p]->n_enriched = D.nb[p];
    }
    // sub-batches of whole instances within the memory budget: about 45% of
    // the free device memory for the per-bucket data of one sub-batch
    size_t mfree = 0, mtotal = 0;
    PM_TRY(hipMemGetInfo(&mfree, &mtotal));
    const size_t budget = (size_t)(0.45 * (double)mfree);
    const size_t per_b = bytes_per_bucket(AL, O.em_iters + 1, t_max, tri != nullptr);
    int p0 = 0;
    while (p0 < P) {
        int p1 = p0;
        size_t used = 0;
        while (p1 < P) {
            const size_t need = (size_t)D.nb[p1] * per_b + (size_t)D.nm[p1] * 4;
            if (p1 > p0 && used + need > budget) break;
            used += need;
            ++p1;
        }
        PM_CALL(run_sub(D, p0, p1, G, Rs, O, tri, st));
        p0 = p1;
    }
    return PM_OK;
}

}  // namespace
}  // namespace pm

using namespace pm;

extern "C" int projection_run(const pm_problem *P, int32_t n_problems, const pm_options *O, pm_result *R)
{
    clear_error();
    if (!P || !O || !R || n_problems < 1) return fail(PM_EINVAL, "need n_problems >= 1 and non-NULL arguments");
    if (O->em_iters < 0 || O->beta < 0) return fail(PM_EINVAL, "need em_iters >= 0 and beta >= 0");
    if (O->precision < PM_FP64 || O->precision > PM_F16) return fail(PM_EINVAL, "unknown precision %d", O->precision);
    const double frac = O->triage_frac > 0 ? O->triage_frac : 0.05;
    if (O->triage && !(frac <= 1)) return fail(PM_EINVAL, "triage_frac must be in (0, 1]");
    hipStream_t st = as_stream(O->stream);
    std::vector<Prepared> Q(n_problems);
    for (int p = 0; p < n_problems; ++p) PM_CALL(prepare(P[p], p, Q[p]));
    TriageModel tri;
    if (O->triage) {
        PM_CALL(read_triage(O->triage_weights, tri));
        for (int p = 0; p < n_problems; ++p)
            if (Q[p].A != 4 || Q[p].l > 21)
                return fail(PM_EINVAL, "problem %d: learned triage is for DNA motifs with l <= 21", p);
    }
    pm_options opt = *O;
    opt.triage_frac = frac;
    if (!O->batched && !O->triage) {
        for (int p = 0; p < n_problems; ++p) PM_CALL(run_single(Q[p], opt, R[p], st));
        return PM_OK;
    }
    if (O->precision == PM_F16)
        for (int p = 0; p < n_problems; ++p)
            if (Q[p].A == 20)
                return fail(PM_EINVAL, "problem %d: the protein matrix-core form runs unbatched (batched = 0)", p);
    // groups of problems sharing alphabet, l, k, s and background, in order of
    // first appearance; unbatched triage runs every problem as its own group
    std::vector<std::vector<int>> groups;
    if (O->batched) {
        std::map<std::tuple<int, int, int, int, std::vector<double>>, int> gid;
        for (int p = 0; p < n_problems; ++p) {
            const auto key = std::make_tuple(Q[p].A, Q[p].l, Q[p].k, Q[p].s, Q[p].bg);
            auto it = gid.find(key);
            if (it == gid.end()) {
                gid.emplace(key, (int)groups.size());
                groups.push_back({p});
            } else {
                groups[it->second].push_back(p);
            }
        }
    } else {
        for (int p = 0; p < n_problems; ++p) groups.push_back({p});
    }
    for (const auto &g : groups) {
        std::vector<const Prepared *> G;
        std::vector<pm_result *> Rs;
        for (int p : g) {
            G.push_back(&Q[p]);
            Rs.push_back(&R[p]);
        }
        PM_CALL(run_group(G, Rs, opt, O->triage ? &tri : nullptr, st));
    }
    return PM_OK;
}

// Sec. 2: the motif length may be a range (l-, l+).  Every length of the range
// is one problem of a single projection_run call (the batched path gives each
// length its own shape class); the paper does not say how lengths compete,
// so the reported choice is the length whose answer has the largest
// log-likelihood ratio per motif column, the longer length on ties (a
// motif's columns each add to the ratio, so the ratio itself favours long
// models fitted to noise; per column it favours the planted motif or a
// piece of it).
extern "C" int projection_run_range(const pm_problem *P, int32_t l_minus, int32_t l_plus, const pm_options *O,
                                    pm_result *R, int32_t *chosen)
{
    clear_error();
    if (!P || !O || !R) return fail(PM_EINVAL, "NULL argument");
    if (l_minus < 1 || l_plus < l_minus || l_plus > 32)
        return fail(PM_EINVAL, "need 1 <= l- <= l+ <= 32 (l- = %d, l+ = %d)", l_minus, l_plus);
    if (P->masks) return fail(PM_EINVAL, "a length range draws its own masks per length (masks must be NULL)");
    if (P->k > l_minus) return fail(PM_EINVAL, "a given k (%d) must not exceed l- (%d)", P->k, l_minus);
    const int n = l_plus - l_minus + 1;
    std::vector<pm_problem> Ps(n, *P);
    for (int q = 0; q < n; ++q) Ps[q].l = l_minus + q;
    PM_CALL(projection_run(Ps.data(), n, O, R));
    int best = -1;
    double bv = -INFINITY;
    for (int q = 0; q < n; ++q) {
        if (R[q].best_trial < 0 || !(R[q].llr == R[q].llr)) continue;
        const double v = R[q].llr / (double)(l_minus + q);
        if (best < 0 || v >= bv) {
            best = q;
            bv = v;
        }
    }
    if (chosen) *chosen = best < 0 ? -1 : l_minus + best;
    return PM_OK;
}
