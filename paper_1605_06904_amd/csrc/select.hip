// a5 (enriched-bucket selection and member lists) and a6 (profiles, theta^0).
//
// The paper finds enriched buckets by comparing every k-mer with every other
// one (Sec. 6, quadratic work) to avoid a |Sigma|^k table.  On MI355X the dense
// counts already sit in HBM (the histogram of projection_hash), so selection is
// a streaming pass: count the passing bins per trial, scan the per-trial
// totals, then one workgroup per trial turns its counts into an LDS bitmap of
// passing keys (one ballot per 64 keys), scans it to give every bucket its
// index and first member slot, and places the member windows with a stable,
// deterministic two-pass counting sort over four window quarters.
#include "pm_common.h"

namespace pm {

struct SelWs {
    int64_t *ne;      // [m] enriched buckets per trial
    int64_t *ms;      // [m] members per trial
    int64_t *bb;      // [m] first bucket of the trial
    int64_t *mb;      // [m] first member slot of the trial
    uint32_t *qcnt;   // [cap_b][4] members of the bucket in each window quarter
    uint32_t *placed; // [cap_b][4] members placed so far by each quarter's wave
};

static SelWs carve(void *ws, int32_t m, int64_t cap_b)
{
    char *p = static_cast<char *>(ws);
    SelWs w;
    w.ne = reinterpret_cast<int64_t *>(p);
    w.ms = w.ne + m;
    w.bb = w.ms + m;
    w.mb = w.bb + m;
    w.qcnt = reinterpret_cast<uint32_t *>(w.mb + m);
    w.placed = w.qcnt + 4 * cap_b;
    return w;
}

struct SelArgs {
    pm_inst one;               // the instance, when inst is NULL
    const pm_inst *inst;       // batch: instance table, or NULL
    const int32_t *item_inst;  // batch: instance of every trial item
    const uint32_t *keys;
    const uint32_t *counts;
    pm_bucket *buckets;
    uint32_t *members;
    int64_t *n_out;
    uint32_t *status;
    SelWs ws;
    int64_t nb, cap_b, cap_m;
    int32_t m;  // trials (items)
    uint32_t s;
    int nwb;  // bitmap words, ceil(nb / 64)
};

__device__ __forceinline__ bool passes(uint32_t c, uint32_t s) { return c >= s && c > 0; }

// per trial: number of passing bins and their total size
__global__ void __launch_bounds__(256) k_sel_count(const SelArgs a)
{
    const int j = blockIdx.x;
    const uint4 *cnt = reinterpret_cast<const uint4 *>(a.counts + (int64_t)j * a.nb);  // nb % 4 == 0
    uint64_t ne = 0, ms = 0;
    for (int64_t b = threadIdx.x; b < a.nb / 4; b += 256) {
        const uint4 v = cnt[b];
        const uint32_t c[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (passes(c[q], a.s)) {
                ne += 1;
                ms += c[q];
            }
    }
    ne = wave_sum(ne);
    ms = wave_sum(ms);
    __shared__ uint64_t red[2][4];
    const int wv = threadIdx.x >> 6;
    if (lane_id() == 0) {
        red[0][wv] = ne;
        red[1][wv] = ms;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a.ws.ne[j] = (int64_t)(red[0][0] + red[0][1] + red[0][2] + red[0][3]);
        a.ws.ms[j] = (int64_t)(red[1][0] + red[1][1] + red[1][2] + red[1][3]);
    }
}

// exclusive scan of per-trial (or per trial-slice) totals, one workgroup:
// bases of every entry, the required totals in n_out, capacity status
__global__ void __launch_bounds__(1024) k_tot_scan(const TotScan a)
{
    __shared__ int64_t sa[1024], sb[1024];
    __shared__ int64_t carry[2];
    if (threadIdx.x == 0) carry[0] = carry[1] = 0;
    __syncthreads();
    for (int64_t base = 0; base < a.n; base += 1024) {
        const int64_t j = base + threadIdx.x;
        const int64_t ve = j < a.n ? a.ne[j] : 0, vm = j < a.n ? a.ms[j] : 0;
        sa[threadIdx.x] = ve;
        sb[threadIdx.x] = vm;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            int64_t ua = 0, ub = 0;
            if ((int)threadIdx.x >= o) {
                ua = sa[threadIdx.x - o];
                ub = sb[threadIdx.x - o];
            }
            __syncthreads();
            sa[threadIdx.x] += ua;
            sb[threadIdx.x] += ub;
            __syncthreads();
        }
        if (j < a.n) {
            a.bb[j] = carry[0] + sa[threadIdx.x] - ve;
            a.mb[j] = carry[1] + sb[threadIdx.x] - vm;
        }
        __syncthreads();
        if (threadIdx.x == 1023) {
            carry[0] += sa[1023];
            carry[1] += sb[1023];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.n_out[0] = carry[0];
        a.n_out[1] = carry[1];
        if ((carry[0] > a.cap_b || carry[1] > a.cap_m) && a.status) atomicOr(a.status, PM_STATUS_CAPACITY);
    }
}

int launch_tot_scan(const TotScan &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_tot_scan, dim3(1), dim3(1024), 0, st, a);
    PM_LAUNCHED();
    return PM_OK;
}

// exclusive prefix sums of n u32 values in place (256 threads, n <= 256 * 64)
__device__ void block_excl_scan(uint32_t *v, int n, uint32_t *tmp)
{
    const int tid = threadIdx.x, per = (n + 255) / 256;
    const int lo = tid * per, hi = lo + per < n ? lo + per : n;
    uint32_t s = 0;
    for (int i = lo; i < hi; ++i) s += v[i];
    tmp[tid] = s;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const uint32_t u = tid >= o ? tmp[tid - o] : 0u;
        __syncthreads();
        tmp[tid] += u;
        __syncthreads();
    }
    uint32_t run = tmp[tid] - s;
    for (int i = lo; i < hi; ++i) {
        const uint32_t x = v[i];
        v[i] = run;
        run += x;
    }
    __syncthreads();
}

// one workgroup (four waves) per trial
__global__ void __launch_bounds__(256) k_sel_emit(const SelArgs a)
{
    extern __shared__ __align__(16) uint64_t bm[];  // [nwb] passing keys
    uint32_t *wcnt = reinterpret_cast<uint32_t *>(bm + a.nwb);  // [nwb] -> buckets before the word
    uint32_t *wsz = wcnt + a.nwb;                               // [nwb] -> members before the word
    __shared__ uint32_t tmp[256];
    const int j = blockIdx.x;
    const int tid = threadIdx.x, wv = tid >> 6, lane = lane_id();
    const uint32_t *cnt = a.counts + (int64_t)j * a.nb;
    const int64_t bbase = a.ws.bb[j], mbase = a.ws.mb[j];
    const pm_inst I = a.inst ? a.inst[a.item_inst[j]] : a.one;

    // ---- bitmap of passing keys, one ballot per word of 64 keys; eight loads
    // in flight per wave
    constexpr int U = 8;
    for (int w0 = wv; w0 < a.nwb; w0 += 4 * U) {
        uint32_t c[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t key = (int64_t)(w0 + 4 * u) * 64 + lane;
            c[u] = (w0 + 4 * u < a.nwb && key < a.nb) ? cnt[key] : 0u;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int wi = w0 + 4 * u;
            const bool flag = passes(c[u], a.s);
            const uint64_t bal = __ballot(flag);
            uint32_t sz = 0;
            if (bal) sz = wave_sum(flag ? c[u] : 0u);
            if (lane == 0 && wi < a.nwb) {
                bm[wi] = bal;
                wcnt[wi] = __popcll(bal);
                wsz[wi] = sz;
            }
        }
    }
    __syncthreads();
    block_excl_scan(wcnt, a.nwb, tmp);
    block_excl_scan(wsz, a.nwb, tmp);

    // ---- bucket records, in key order
    for (int wi = tid; wi < a.nwb; wi += 256) {
        uint64_t bits = bm[wi];
        int64_t b = bbase + wcnt[wi];
        int64_t first = mbase + wsz[wi];
        while (bits) {
            const int bit = __ffsll((unsigned long long)bits) - 1;
            bits &= bits - 1;
            const int64_t key = (int64_t)wi * 64 + bit;
            const uint32_t c = cnt[key];
            if (b < a.cap_b) {
                pm_bucket *B = a.buckets + b;
                st_agent(&B->trial, (uint32_t)j);
                st_agent(&B->key, (uint32_t)key);
                st_agent(&B->size, c);
                st_agent(&B->first, (uint32_t)first);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    st_agent(a.ws.qcnt + 4 * b + q, 0u);
                    st_agent(a.ws.placed + 4 * b + q, 0u);
                }
            }
            ++b;
            first += c;
        }
    }
    // the records, counters and first slots above are agent-scope atomics read
    // back only by this workgroup: a workgroup barrier orders them (an
    // agent-scope fence would write back and invalidate the whole L2)
    __syncthreads();

    // ---- members: wave wv owns windows [lo, hi); pass 0 counts per bucket,
    // pass 1 places them after the members of earlier quarters
    const uint32_t *kj = a.keys + I.key_base + (int64_t)(j - I.first_item) * I.x;
    const int64_t lo = I.x * wv / 4, hi = I.x * (wv + 1) / 4;
    for (int pass = 0; pass < 2; ++pass) {
        for (int64_t wb = lo; wb < hi; wb += 64 * U) {
          uint32_t kk[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
              const int64_t w = wb + 64 * u + lane;
              kk[u] = w < hi ? kj[w] : 0u;
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int64_t w = wb + 64 * u + lane;
            const bool valid = w < hi;
            const uint32_t key = kk[u];
            const bool flag = valid && key < a.nb && ((bm[key >> 6] >> (key & 63)) & 1ull);
            uint64_t bal = __ballot(flag);
            while (bal) {
                const int leader = __ffsll((unsigned long long)bal) - 1;
                const uint32_t lk = __shfl(key, leader);
                const bool peer = flag && key == lk;
                const uint64_t peers = __ballot(peer);
                int64_t slot0 = -1;
                if (lane == leader) {
                    const uint64_t word = bm[lk >> 6];
                    const int64_t b = bbase + wcnt[lk >> 6] + __popcll(word & ((1ull << (lk & 63)) - 1ull));
                    if (b < a.cap_b) {
                        if (pass == 0) {
                            atomicAdd(a.ws.qcnt + 4 * b + wv, (uint32_t)__popcll(peers));
                        } else {
                            int64_t base = ld_agent(&a.buckets[b].first);
                            for (int q = 0; q < wv; ++q) base += ld_agent(a.ws.qcnt + 4 * b + q);
                            slot0 = base + atomicAdd(a.ws.placed + 4 * b + wv, (uint32_t)__popcll(peers));
                        }
                    }
                }
                if (pass == 1) {
                    slot0 = __shfl(slot0, leader);
                    if (peer && slot0 >= 0) {
                        const int64_t slot = slot0 + __popcll(peers & lanemask_lt());
                        if (slot < a.cap_m) a.members[slot] = (uint32_t)w;
                    }
                }
                bal &= ~peers;
            }
          }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- a6
struct ProfArgs {
    pm_inst one;               // the instance, when inst is NULL
    const pm_inst *inst;       // batch: instance table, or NULL
    const int32_t *item_inst;  // batch: instance of every trial item
    const pm_bucket *buckets;
    const uint32_t *members;
    const int64_t *n_dev;
    uint32_t *profile;
    int64_t B, cap_m;
    int l, A;
};

// one wave per bucket; lane p owns column p
__global__ void __launch_bounds__(256) k_profile(const ProfArgs a)
{
    __shared__ uint32_t cnt[4][20 * 32];
    const int wv = threadIdx.x >> 6, lane = lane_id();
    const int64_t b = (int64_t)blockIdx.x * 4 + wv;
    int64_t nvalid = a.n_dev ? *a.n_dev : a.B;
    if (nvalid > a.B) nvalid = a.B;
    if (b >= nvalid) return;
    uint32_t *C = cnt[wv];
    for (int i = lane; i < a.A * 32; i += 64) C[i] = 0;
    const pm_bucket bk = a.buckets[b];
    const pm_inst I = a.inst ? a.inst[a.item_inst[bk.trial]] : a.one;
    const int64_t lm1 = a.l - 1;
    const uint32_t size = (int64_t)bk.first + bk.size <= a.cap_m ? bk.size : 0u;
    // up to 64 members at a time: lane r finds where member r starts, then
    // every column lane reads the members' symbols one after another
    for (uint32_t r0 = 0; r0 < size; r0 += 64) {
        const uint32_t nr = size - r0 < 64u ? size - r0 : 64u;
        int64_t Pm = 0;
        if ((uint32_t)lane < nr) {
            const int64_t w = a.members[(int64_t)bk.first + r0 + lane];
            int lo = 0, hi = I.t;  // last sequence whose first window <= w
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (I.offsets[mid] - (int64_t)mid * lm1 <= w) lo = mid;
                else hi = mid;
            }
            Pm = w + (int64_t)lo * lm1;
        }
        for (uint32_t r = 0; r < nr; ++r) {
            const int64_t P = __shfl(Pm, (int)r);
            if (lane < a.l) {
                const uint32_t code = a.A == 4 ? dna_sym(I.packed, P + lane) : prot_sym(I.packed, P + lane);
                C[code * 32 + lane] += 1;
            }
        }
    }
    uint32_t *out = a.profile + b * a.A * a.l;
    for (int i = lane; i < a.A * a.l; i += 64) out[i] = C[(i / a.l) * 32 + (i % a.l)];
}

// one thread per (bucket, column): the bucket's size from column 0, then the
// column's A letters
__global__ void k_theta_init(const uint32_t *__restrict__ prof, const int64_t *n_dev, int64_t B, int A,
                             int l, const double *__restrict__ bg, double beta, double *__restrict__ th)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t b = g <= 0xffffffffll ? (int64_t)((uint32_t)g / (uint32_t)l) : g / l;
    int64_t nvalid = n_dev ? *n_dev : B;
    if (nvalid > B) nvalid = B;
    if (b >= nvalid) return;
    const int p = (int)(g - b * l);
    const int64_t per = (int64_t)A * l;
    const uint32_t *P = prof + b * per;
    double *T = th + b * per;
    double size = 0;
    for (int cc = 0; cc < A; ++cc) size += P[cc * l];
    for (int c = 0; c < A; ++c) T[c * l + p] = (P[c * l + p] + beta * bg[c]) / (size + beta);
}

}  // namespace pm

using namespace pm;

extern "C" size_t pm_select_workspace(int32_t m, int64_t cap_buckets)
{
    if (m < 0 || cap_buckets < 0) return 0;
    return (size_t)m * 4 * sizeof(int64_t) + (size_t)cap_buckets * 8 * sizeof(uint32_t) + 256;
}

static int select_launch(SelArgs &a, int A, int k, hipStream_t st)
{
    if (ipow(A, k) > (1ll << 19)) return fail(PM_ERANGE, "|Sigma|^k above 2^19");
    a.nb = ipow(A, k);
    hipLaunchKernelGGL(k_sel_count, dim3(a.m), dim3(256), 0, st, a);
    PM_LAUNCHED();
    const TotScan ts{a.ws.ne, a.ws.ms, a.ws.bb, a.ws.mb, a.m, a.cap_b, a.cap_m, a.n_out, a.status};
    if (int rc = launch_tot_scan(ts, st)) return rc;
    a.nwb = (int)((a.nb + 63) / 64);
    const size_t lds = (size_t)a.nwb * 16;
    static bool attr = false;
    if (!attr) {
        // the kernel also holds 1 KB of static LDS
        (void)hipFuncSetAttribute((const void *)k_sel_emit, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  device_lds_bytes() - 2048);
        (void)hipGetLastError();  // an unsupported attribute must not poison the launch check
        attr = true;
    }
    hipLaunchKernelGGL(k_sel_emit, dim3(a.m), dim3(256), lds, st, a);
    PM_LAUNCHED();
    return PM_OK;
}

static int check_select_args(int32_t items, const uint32_t *keys, const uint32_t *counts, const int64_t *n_out,
                             void *ws, size_t ws_bytes, pm_bucket *buckets, int64_t cap_buckets,
                             uint32_t *members, int64_t cap_members)
{
    if (items < 1) return fail(PM_EINVAL, "m must be >= 1");
    if (!keys || !counts || !n_out || !ws) return fail(PM_EINVAL, "keys, counts, n_out and ws are required");
    if (cap_buckets < 0 || cap_members < 0) return fail(PM_EINVAL, "negative capacity");
    if ((cap_buckets > 0 && !buckets) || (cap_members > 0 && !members))
        return fail(PM_EINVAL, "NULL output with a non-zero capacity");
    if (cap_members > 0xffffffffll) return fail(PM_ERANGE, "cap_members must be below 2^32");
    if (ws_bytes < pm_select_workspace(items, cap_buckets)) return fail(PM_EINVAL, "workspace too small");
    return PM_OK;
}

extern "C" int bucket_select(const pm_seqs *S, int32_t l, int32_t k, const uint32_t *keys,
                             const uint32_t *counts, int32_t m, uint32_t s, pm_bucket *buckets,
                             int64_t cap_buckets, uint32_t *members, int64_t cap_members,
                             int64_t *n_out, void *ws, size_t ws_bytes, uint32_t *status, void *stream)
{
    clear_error();
    int rc = check_seqs(S, l);
    if (rc) return rc;
    if (k < 1 || k > l) return fail(PM_EINVAL, "need 1 <= k <= l");
    if ((rc = check_select_args(m, keys, counts, n_out, ws, ws_bytes, buckets, cap_buckets, members, cap_members)))
        return rc;
    SelArgs a{};
    a.one = inst_of(S, l);
    a.keys = keys;
    a.counts = counts;
    a.buckets = buckets;
    a.members = members;
    a.n_out = n_out;
    a.status = status;
    a.ws = carve(ws, m, cap_buckets);
    a.cap_b = cap_buckets;
    a.cap_m = cap_members;
    a.m = m;
    a.s = s;
    return select_launch(a, S->alphabet, k, as_stream(stream));
}

extern "C" int bucket_select_batch(const pm_batch *B, const uint32_t *keys, const uint32_t *counts, uint32_t s,
                                   pm_bucket *buckets, int64_t cap_buckets, uint32_t *members,
                                   int64_t cap_members, int64_t *n_out, void *ws, size_t ws_bytes,
                                   uint32_t *status, void *stream)
{
    clear_error();
    int rc = check_batch(B, nullptr);
    if (rc) return rc;
    if ((rc = check_select_args(B->items, keys, counts, n_out, ws, ws_bytes, buckets, cap_buckets, members,
                                cap_members)))
        return rc;
    SelArgs a{};
    a.inst = B->inst;
    a.item_inst = B->item_inst;
    a.keys = keys;
    a.counts = counts;
    a.buckets = buckets;
    a.members = members;
    a.n_out = n_out;
    a.status = status;
    a.ws = carve(ws, B->items, cap_buckets);
    a.cap_b = cap_buckets;
    a.cap_m = cap_members;
    a.m = B->items;
    a.s = s;
    return select_launch(a, B->alphabet, B->k, as_stream(stream));
}

static int profile_launch(const ProfArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_profile, dim3((unsigned)((a.B + 3) / 4)), dim3(256), 0, st, a);
    PM_LAUNCHED();
    return PM_OK;
}

extern "C" int bucket_profile(const pm_seqs *S, int32_t l, const pm_bucket *buckets,
                              const uint32_t *members, int64_t cap_members, int64_t B,
                              const int64_t *n_dev, uint32_t *profile, void *stream)
{
    clear_error();
    int rc = check_seqs(S, l);
    if (rc) return rc;
    if (B < 0) return fail(PM_EINVAL, "B must be >= 0");
    if (B == 0) return PM_OK;
    if (!buckets || !members || !profile) return fail(PM_EINVAL, "NULL buffer");
    ProfArgs a{};
    a.one = inst_of(S, l);
    a.buckets = buckets;
    a.members = members;
    a.n_dev = n_dev;
    a.profile = profile;
    a.B = B;
    a.cap_m = cap_members;
    a.l = l;
    a.A = S->alphabet;
    return profile_launch(a, as_stream(stream));
}

extern "C" int bucket_profile_batch(const pm_batch *Bt, const pm_bucket *buckets, const uint32_t *members,
                                    int64_t cap_members, int64_t B, const int64_t *n_dev, uint32_t *profile,
                                    void *stream)
{
    clear_error();
    int rc = check_batch(Bt, nullptr);
    if (rc) return rc;
    if (B < 0) return fail(PM_EINVAL, "B must be >= 0");
    if (B == 0) return PM_OK;
    if (!buckets || !members || !profile) return fail(PM_EINVAL, "NULL buffer");
    ProfArgs a{};
    a.inst = Bt->inst;
    a.item_inst = Bt->item_inst;
    a.buckets = buckets;
    a.members = members;
    a.n_dev = n_dev;
    a.profile = profile;
    a.B = B;
    a.cap_m = cap_members;
    a.l = Bt->l;
    a.A = Bt->alphabet;
    return profile_launch(a, as_stream(stream));
}

extern "C" int theta_init(int32_t alphabet, int32_t l, const uint32_t *profile, int64_t B,
                          const int64_t *n_dev, const double *bg, double beta, double *theta0,
                          void *stream)
{
    clear_error();
    if (alphabet != 4 && alphabet != 20) return fail(PM_EINVAL, "alphabet must be 4 or 20");
    if (l < 1 || l > 32) return fail(PM_EINVAL, "need 1 <= l <= 32");
    if (B < 0 || beta < 0) return fail(PM_EINVAL, "need B >= 0 and beta >= 0");
    if (B == 0) return PM_OK;
    if (!profile || !bg || !theta0) return fail(PM_EINVAL, "NULL buffer");
    const int64_t total = B * l;
    const int threads = 256;
    hipLaunchKernelGGL(k_theta_init, dim3((unsigned)((total + threads - 1) / threads)), dim3(threads), 0,
                       as_stream(stream), profile, n_dev, B, alphabet, l, bg, beta, theta0);
    PM_LAUNCHED();
    return PM_OK;
}
