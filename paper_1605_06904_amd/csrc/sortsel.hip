// a3 + a4 + a5 without a count table: enriched buckets of key spaces too
// large for LDS histograms (DNA k up to 16, protein k up to 7).
//
// Alg. 2 step 3 defines a bucket by the l-mers that share a projected k-mer
// and keeps it when it holds at least s of them (Sec. 6).  The |Sigma|^k
// table of PROJECTION1 (Sec. 5.2) stops fitting on-chip long before keys stop
// fitting 32 bits; the paper's own answer to that space problem is its K2
// kernel (Sec. 6: every l-mer compared with every other, O(x^2) work).  Here
// a trial's buckets come from sorting instead: one workgroup owns one
// (trial, key-range slice), counts the slice's keys in a coarse LDS histogram
// of 4096 key ranges, takes the leading ranges whose windows fit an LDS
// buffer of 8192 (key, window) pairs, gathers those pairs, sorts them with a
// bitonic network, and reads buckets off the runs of equal keys, in key order
// with members in window order -- the same lists as the count-table path.
// A range with more windows than the buffer holds is narrowed (finer coarse
// bins) until it is a single key, which then forms its bucket directly.
// Nothing but the bucket records and members reaches HBM; like the fused
// count-table path, one pass counts (per-slice totals, scanned on the device)
// and a second identical pass writes.
#include "hash_dev.h"

namespace pm {

constexpr int kSortCap = 8192;     // (key, window) pairs sorted at once
constexpr int kCoarseBins = 4096;  // key ranges of the coarse histogram
constexpr int kCtlWords = 64;      // block-scan partials and round state
constexpr int kSortWaves = kHashThreads / kWave;

struct HsortArgs {
    HashArgs h;
    uint32_t s;
    uint64_t slice_width;           // keys per slice (the last one may be shorter)
    int64_t *tot_b, *tot_m;         // [items * nslices]
    const int64_t *base_b, *base_m; // [items * nslices] (EMIT)
    pm_bucket *buckets;
    uint32_t *members;
    int64_t cap_b, cap_m;
};

// Exclusive prefix of (a, b) over the workgroup's threads, in thread order;
// tot_* receive the workgroup totals.  ctl holds 2 * kSortWaves words.
__device__ __forceinline__ void block_excl_scan2(uint32_t &a, uint32_t &b, uint32_t *ctl, uint32_t &tot_a,
                                                 uint32_t &tot_b)
{
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    const uint32_t ia = wave_incl_scan(a), ib = wave_incl_scan(b);
    if (lane == kWave - 1) {
        ctl[2 * wave] = ia;
        ctl[2 * wave + 1] = ib;
    }
    __syncthreads();
    uint32_t pa = 0, pb = 0, sa = 0, sb = 0;
    for (int w = 0; w < kSortWaves; ++w) {
        const uint32_t va = ctl[2 * w], vb = ctl[2 * w + 1];
        if (w < wave) {
            pa += va;
            pb += vb;
        }
        sa += va;
        sb += vb;
    }
    a = pa + ia - a;
    b = pb + ib - b;
    tot_a = sa;
    tot_b = sb;
    __syncthreads();
}

// smallest shift whose 2^sh-wide bins cover `range` keys in kCoarseBins bins
__device__ __forceinline__ int coarse_shift(uint64_t range)
{
    int sh = 0;
    while (((range + (1ull << sh) - 1) >> sh) > (uint64_t)kCoarseBins) ++sh;
    return sh;
}

template <int A, int K, bool EMIT>
__global__ void __launch_bounds__(kHashThreads) k_hsort(const HsortArgs g)
{
    const HashArgs &a = g.h;
    extern __shared__ __align__(16) uint32_t smem[];
    const int slice = blockIdx.x % a.nslices;
    const int j = blockIdx.x / a.nslices;
    const int tid = threadIdx.x;
    const int64_t e = (int64_t)blockIdx.x;  // (item, slice) entry

    const uint32_t mask = a.masks[j];
    if (!mask_ok(a, mask)) {
        if (tid == 0) {
            if (slice == 0 && a.status) atomicOr(a.status, PM_STATUS_BAD_MASK);
            if (!EMIT) g.tot_b[e] = g.tot_m[e] = 0;
        }
        return;
    }
    uint64_t *buf = reinterpret_cast<uint64_t *>(smem);  // [kSortCap]
    uint32_t *hist = smem + 2 * kSortCap;                 // [kCoarseBins]
    uint32_t *ctl = hist + kCoarseBins;                   // [kCtlWords]
    uint32_t *seq = ctl + kCtlWords;
    int32_t *wst = reinterpret_cast<int32_t *>(seq + a.seq_cap);
    const Staged st = stage_input<A>(a, j, seq, wst);
    int pos[K];
    kept_positions<A, K>(mask, pos);
    const int64_t x = st.I.x;
    const uint64_t s_lo = (uint64_t)slice * g.slice_width;
    const uint64_t s_hi = min((uint64_t)a.nb, s_lo + g.slice_width);
    const int sh0 = coarse_shift(s_hi > s_lo ? s_hi - s_lo : 1);
    const int64_t bb = EMIT ? g.base_b[e] : 0, mb = EMIT ? g.base_m[e] : 0;
    int64_t rb = 0, rm = 0;  // buckets and members of this entry so far
    uint64_t lo = s_lo;
    int sh = sh0;
    __syncthreads();

    while (lo < s_hi) {
        const uint64_t r_hi = min(s_hi, lo + ((uint64_t)kCoarseBins << sh));
        const uint32_t nbins = (uint32_t)((r_hi - lo + (1ull << sh) - 1) >> sh);
        // 1. coarse histogram of the keys in [lo, r_hi)
        for (int b = tid; b < kCoarseBins; b += kHashThreads) hist[b] = 0;
        if (tid == 0) ctl[2 * kSortWaves] = 0xffffffffu;
        __syncthreads();
        {
            int i = 0;
            for (int64_t w = tid; w < x; w += kHashThreads) {
                const uint64_t key = window_key<A, K>(a, st, pos, w, i);
                if (key >= lo && key < r_hi) atomicAdd(hist + (uint32_t)((key - lo) >> sh), 1u);
            }
        }
        __syncthreads();
        // 2. the leading bins whose windows fit the sort buffer
        constexpr int kPer = kCoarseBins / kHashThreads;
        uint32_t c[kPer], sum = 0;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            c[q] = hist[tid * kPer + q];
            sum += c[q];
        }
        uint32_t excl = sum, dummy = 0, total = 0, dtot = 0;
        block_excl_scan2(excl, dummy, ctl, total, dtot);
        {
            uint32_t run = excl;
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                run += c[q];
                if (run > (uint32_t)kSortCap) {
                    atomicMin(ctl + 2 * kSortWaves, (uint32_t)(tid * kPer + q));
                    break;
                }
            }
        }
        __syncthreads();
        const uint32_t first_over = ctl[2 * kSortWaves];
        const uint32_t take = min(first_over, nbins);
        // windows in the taken bins: the prefix up to bin `take`
        if (tid == 0) ctl[2 * kSortWaves + 1] = 0;
        __syncthreads();
        {
            uint32_t run = excl;
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                const uint32_t b = tid * kPer + q;
                if (b < take) run += c[q];
            }
            if (tid * kPer < take && (tid + 1) * kPer >= take) ctl[2 * kSortWaves + 1] = run;
        }
        __syncthreads();
        const uint32_t n = take > 0 ? ctl[2 * kSortWaves + 1] : 0;
        const uint32_t c_first = hist[0];
        __syncthreads();

        if (take == 0) {
            if (sh > 0) {  // the first bin alone is too large: look at it in finer bins
                sh = sh > 12 ? sh - 12 : 0;
                continue;
            }
            // a single key with more windows than the buffer: its own bucket,
            // members in window order by an ordered compaction
            if (c_first >= g.s) {
                if (EMIT) {
                    const int64_t idx = bb + rb;
                    if (tid == 0 && idx < g.cap_b)
                        g.buckets[idx] = pm_bucket{(uint32_t)j, (uint32_t)lo, c_first, (uint32_t)(mb + rm)};
                    int i = 0;
                    uint32_t placed = 0;
                    for (int64_t w0 = 0; w0 < x; w0 += kHashThreads) {
                        const int64_t w = w0 + tid;
                        const bool hit = w < x && window_key<A, K>(a, st, pos, w, i) == lo;
                        uint32_t f = hit ? 1u : 0u, d0 = 0, tot = 0, d1 = 0;
                        block_excl_scan2(f, d0, ctl, tot, d1);
                        const int64_t ms = mb + rm + placed + f;
                        if (hit && ms < g.cap_m) g.members[ms] = (uint32_t)w;
                        placed += tot;
                    }
                }
                rb += 1;
                rm += c_first;
            }
            lo += 1;
            sh = sh0;
            continue;
        }
        const uint64_t hi = min(r_hi, lo + ((uint64_t)take << sh));
        if (n > 0) {
            // 3. gather the (key, window) pairs of [lo, hi) and sort them
            if (tid == 0) ctl[2 * kSortWaves + 2] = 0;
            __syncthreads();
            {
                int i = 0;
                for (int64_t w = tid; w < x; w += kHashThreads) {
                    const uint64_t key = window_key<A, K>(a, st, pos, w, i);
                    if (key >= lo && key < hi) {
                        const uint32_t slot = atomicAdd(ctl + 2 * kSortWaves + 2, 1u);
                        buf[slot] = (key << 32) | (uint64_t)w;
                    }
                }
            }
            uint32_t P = 64;
            while (P < n) P <<= 1;
            for (uint32_t q = n + tid; q < P; q += kHashThreads) buf[q] = ~0ull;
            __syncthreads();
            for (uint32_t kk = 2; kk <= P; kk <<= 1) {
                for (uint32_t jj = kk >> 1; jj > 0; jj >>= 1) {
                    for (uint32_t q = tid; q < P / 2; q += kHashThreads) {
                        const uint32_t i0 = ((q & ~(jj - 1)) << 1) | (q & (jj - 1));
                        const uint32_t i1 = i0 | jj;
                        const uint64_t u = buf[i0], v = buf[i1];
                        const bool up = (i0 & kk) == 0;
                        if ((u > v) == up) {
                            buf[i0] = v;
                            buf[i1] = u;
                        }
                    }
                    __syncthreads();
                }
            }
            // 4. runs of equal keys, in order; each thread starts the runs that
            // begin in its chunk
            const uint32_t chunk = (n + kHashThreads - 1) / kHashThreads;
            const uint32_t c0 = min(n, tid * chunk), c1 = min(n, c0 + chunk);
            uint32_t nbk = 0, nmem = 0;
            for (uint32_t q = c0; q < c1; ++q) {
                const uint32_t key = (uint32_t)(buf[q] >> 32);
                if (q > 0 && (uint32_t)(buf[q - 1] >> 32) == key) continue;
                uint32_t len = 1;
                while (q + len < n && (uint32_t)(buf[q + len] >> 32) == key) ++len;
                if (len >= g.s) {
                    nbk += 1;
                    nmem += len;
                }
            }
            uint32_t bi = nbk, mi = nmem, tb = 0, tm = 0;
            block_excl_scan2(bi, mi, ctl, tb, tm);
            if (EMIT) {
                for (uint32_t q = c0; q < c1; ++q) {
                    const uint32_t key = (uint32_t)(buf[q] >> 32);
                    if (q > 0 && (uint32_t)(buf[q - 1] >> 32) == key) continue;
                    uint32_t len = 1;
                    while (q + len < n && (uint32_t)(buf[q + len] >> 32) == key) ++len;
                    if (len < g.s) continue;
                    const int64_t idx = bb + rb + bi;
                    const int64_t first = mb + rm + mi;
                    if (idx < g.cap_b) g.buckets[idx] = pm_bucket{(uint32_t)j, key, len, (uint32_t)first};
                    for (uint32_t r = 0; r < len; ++r)
                        if (first + r < g.cap_m) g.members[first + r] = (uint32_t)buf[q + r];
                    bi += 1;
                    mi += len;
                }
            }
            rb += tb;
            rm += tm;
            __syncthreads();
        }
        lo = hi;
        sh = sh0;
    }
    if (!EMIT && tid == 0) {
        g.tot_b[e] = rb;
        g.tot_m[e] = rm;
    }
}

template <int A, int K, bool EMIT>
static int launch_hsort(const HsortArgs &g, size_t lds, int blocks, hipStream_t st)
{
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)k_hsort<A, K, EMIT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  device_lds_bytes());
        (void)hipGetLastError();
        attr_set = true;
    }
    hipLaunchKernelGGL((k_hsort<A, K, EMIT>), dim3(blocks), dim3(kHashThreads), lds, st, g);
    PM_LAUNCHED();
    return PM_OK;
}

// run-time (alphabet, k) -> compile-time kernel: DNA k 8..16, protein k 4..7
template <int K>
static int dispatch_hsort(int alphabet, int k, bool emit, const HsortArgs &g, size_t lds, int blocks, hipStream_t st)
{
    if constexpr (K > 16) {
        return fail(PM_ERANGE, "k=%d not supported by the sorted selection", k);
    } else {
        if (k != K) return dispatch_hsort<K + 1>(alphabet, k, emit, g, lds, blocks, st);
        if (alphabet == 4) {
            if constexpr (K >= kSortKMinDna)
                return emit ? launch_hsort<4, K, true>(g, lds, blocks, st) : launch_hsort<4, K, false>(g, lds, blocks, st);
            return fail(PM_ERANGE, "k=%d below the sorted selection's range for DNA", k);
        }
        if constexpr (K >= kSortKMinProt && K <= 7)
            return emit ? launch_hsort<20, K, true>(g, lds, blocks, st) : launch_hsort<20, K, false>(g, lds, blocks, st);
        return fail(PM_ERANGE, "k=%d outside the sorted selection's range for protein", k);
    }
}

// LDS bytes and slices for the largest instance; 0 after fail()
static size_t hsort_layout(HashArgs &a, int64_t x_max, int64_t nw_max, int t_max)
{
    const int lds_max = device_lds_bytes();
    const int64_t sw = staged_words(a.A, nw_max);
    a.off_cap = (t_max + 1) * 4 <= 8 * 1024 ? t_max + 1 : 0;
    a.seq_cap = sw * 4 <= 48 * 1024 && (a.A == 4 || a.off_cap) ? (int)sw : 0;
    a.hist_words = 0;
    a.slice_bins = 0;
    // slices of the key range sized for about half a sort buffer of windows
    // each when keys spread evenly
    int64_t ns = (2 * x_max + kSortCap - 1) / kSortCap;
    if (ns < 1) ns = 1;
    if (ns > a.nb) ns = a.nb;
    a.nslices = (int)ns;
    const size_t bytes = (size_t)(2 * kSortCap + kCoarseBins + kCtlWords + a.seq_cap + a.off_cap) * 4;
    if ((int64_t)bytes > lds_max) {
        fail(PM_ERANGE, "input too large for the sorted selection's LDS budget");
        return 0;
    }
    return bytes;
}

static size_t hsort_ws_bytes(int64_t entries) { return entries < 0 ? 0 : (size_t)entries * 4 * sizeof(int64_t) + 256; }

static int64_t hsort_entries(HashArgs a, int32_t items, int64_t x_max, int64_t nw_max, int t_max)
{
    if (!hsort_layout(a, x_max, nw_max, t_max)) return -1;
    return (int64_t)items * a.nslices;
}

int hsort_check_k(int A, int k)
{
    if (A == 4 && (k < kSortKMinDna || k > 16))
        return fail(PM_ERANGE, "the sorted selection takes DNA k from %d to 16 (k=%d)", kSortKMinDna, k);
    if (A == 20 && (k < kSortKMinProt || k > 7))
        return fail(PM_ERANGE, "the sorted selection takes protein k from %d to 7 (k=%d)", kSortKMinProt, k);
    return PM_OK;
}

size_t hsort_workspace(int A, int l, int k, int32_t items, int64_t x_max, int64_t nw_max, int t_max)
{
    HashArgs a{};
    a.A = A;
    a.nb = ipow(A, k);
    a.l = l;
    a.k = k;
    return hsort_ws_bytes(hsort_entries(a, items, x_max, nw_max, t_max));
}

int hsort_run(HashArgs &a, int A, int32_t items, int64_t x_max, int64_t nw_max, int t_max, uint32_t s,
              pm_bucket *buckets, int64_t cap_b, uint32_t *members, int64_t cap_m, int64_t *n_out, void *ws,
              size_t ws_bytes, hipStream_t st)
{
    if (int rc = hsort_check_k(A, a.k)) return rc;
    const size_t lds = hsort_layout(a, x_max, nw_max, t_max);
    if (!lds) return PM_ERANGE;
    if (x_max >= (int64_t)1 << 31) return fail(PM_ERANGE, "more than 2^31 windows in one instance");
    const int64_t entries = (int64_t)items * a.nslices;
    if (entries > 0x7fffffff) return fail(PM_ERANGE, "too many trials x slices");
    if (ws_bytes < hsort_ws_bytes(entries))
        return fail(PM_EINVAL, "workspace of %zu bytes, need %zu", ws_bytes, hsort_ws_bytes(entries));
    if (((uintptr_t)ws & 7) != 0) return fail(PM_EINVAL, "workspace must be 8-byte aligned");
    int64_t *w = static_cast<int64_t *>(ws);
    HsortArgs g{};
    g.h = a;
    g.s = s;
    g.slice_width = ((uint64_t)a.nb + a.nslices - 1) / a.nslices;
    g.tot_b = w;
    g.tot_m = w + entries;
    g.base_b = w + 2 * entries;
    g.base_m = w + 3 * entries;
    g.buckets = buckets;
    g.members = members;
    g.cap_b = cap_b;
    g.cap_m = cap_m;
    if (int rc = dispatch_hsort<1>(A, a.k, false, g, lds, (int)entries, st)) return rc;
    const TotScan ts{g.tot_b, g.tot_m, w + 2 * entries, w + 3 * entries, entries, cap_b, cap_m, n_out, a.status};
    if (int rc = launch_tot_scan(ts, st)) return rc;
    if (cap_b == 0 && cap_m == 0) return PM_OK;  // sizing only
    return dispatch_hsort<1>(A, a.k, true, g, lds, (int)entries, st);
}

}  // namespace pm
