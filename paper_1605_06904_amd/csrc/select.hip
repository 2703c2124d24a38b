// a5 (enriched-bucket selection and member lists) and a6 (profiles, theta^0).
//
// The paper finds enriched buckets by comparing every k-mer with every other
// one (Sec. 6, quadratic work) to avoid a |Sigma|^k table.  On MI355X the dense
// counts already sit in HBM (the histogram of projection_hash), so selection
// reads them once: a counting pass per trial writes the number of passing
// bins, their total size and a bitmap of the passing keys (one bit per key);
// projection_hash_select has its hash kernel write these instead.  After a
// scan of the per-trial totals, one workgroup per trial loads its bitmap into
// LDS, gathers the counts of the passing keys only, scans them into bucket
// numbers and first member slots, and places the member windows in window
// order.  A trial of few members lists its passing windows per wave quarter
// in LDS and places them from the lists; otherwise a stable counting sort
// goes over the windows in chunks: per-wave counts by LDS atomics, then each
// wave groups its passing windows by key (by ballots over the key bits when
// many pass), every bucket keeping its next free slot per wave in LDS.
#include <algorithm>

#include "pm_common.h"

namespace pm {

struct SelWs {
    int64_t *ne;      // [m] enriched buckets per trial
    int64_t *ms;      // [m] members per trial
    int64_t *bb;      // [m] first bucket of the trial
    int64_t *mb;      // [m] first member slot of the trial
    int64_t *n_heavy; // [1] trials with more buckets than the first emit launch takes
    int64_t *qctr;    // [4] next unit of each heavy launch (work queue heads, [0..2]), then
                      // the most buckets of a heavy trial ([3], written by the scan)
    int32_t *heavy;   // [m] those trials, in order
    int64_t *nep;     // [m][parts] buckets of each part of a trial's bins (parts > 1)
    int64_t *msp;     // [m][parts] their members
    uint64_t *bits;   // [m][nwb] passing keys: bit key % 64 of word key / 64
};

// parts of a trial's bins counted by separate workgroups: enough workgroups
// (about 16 384) that the launch does not end on a partly filled wave of
// them, each part at least 32 bitmap words
static int sel_parts(int32_t m, int64_t nwb)
{
    int64_t p = (16384 + (int64_t)m - 1) / std::max<int64_t>(m, 1);
    p = std::min<int64_t>(p, std::max<int64_t>(1, nwb / 32));
    return (int)std::max<int64_t>(1, std::min<int64_t>(p, 64));
}

static size_t sel_head_bytes(int32_t m, int64_t nwb)
{
    return (size_t)m * 4 * sizeof(int64_t) + 5 * sizeof(int64_t) + (((size_t)m * 4 + 7) & ~(size_t)7) +
           (size_t)m * sel_parts(m, nwb) * 2 * sizeof(int64_t);
}

static size_t sel_ws_bytes(int32_t m, int64_t nwb)
{
    return sel_head_bytes(m, nwb) + (size_t)m * nwb * 8 + 256;
}

static SelWs carve(void *ws, int32_t m, int64_t nwb)
{
    char *p = static_cast<char *>(ws);
    SelWs w;
    w.ne = reinterpret_cast<int64_t *>(p);
    w.ms = w.ne + m;
    w.bb = w.ms + m;
    w.mb = w.bb + m;
    w.n_heavy = w.mb + m;
    w.qctr = w.n_heavy + 1;
    w.heavy = reinterpret_cast<int32_t *>(w.qctr + 4);
    w.nep = reinterpret_cast<int64_t *>(p + (size_t)m * 4 * sizeof(int64_t) + 5 * sizeof(int64_t) +
                                        (((size_t)m * 4 + 7) & ~(size_t)7));
    w.msp = w.nep + (int64_t)m * sel_parts(m, nwb);
    w.bits = reinterpret_cast<uint64_t *>(p + sel_head_bytes(m, nwb));
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
    int64_t take_lo, take_hi;  // the trials a launch takes: take_lo < buckets <= take_hi
    int32_t m;                 // trials (items)
    uint32_t s;
    int nwb;    // bitmap words, ceil(nb / 64)
    int cb;     // buckets whose cursors the LDS holds
    int parts;  // k_sel_count: workgroups per trial
    int ranges; // k_sel_emit_heavy: bucket ranges of cb per trial at most
    int tier;   // k_sel_emit_heavy: its work queue (ws.qctr[tier])
};

// per (trial, part of its bins): number of passing bins, their total size
// and the bitmap words of the passing keys.  Lane i of a wave reads bins 4i ..
// 4i+3 of 256 as one 16-byte load, and the four ballots (one per bin of the
// load) become four words in lane-major order: bit 16q + i of word g is bin
// 64g + 4i + q.  The emit pass puts the words in key order.
__global__ void __launch_bounds__(256) k_sel_count(const SelArgs a)
{
    const int j = blockIdx.x / a.parts, part = blockIdx.x % a.parts;
    const int wv = threadIdx.x >> 6, lane = lane_id();
    const uint4 *cnt = reinterpret_cast<const uint4 *>(a.counts + (int64_t)j * a.nb);  // nb % 4 == 0
    uint64_t *bits = a.ws.bits + (int64_t)j * a.nwb;
    const uint32_t smin = a.s > 1u ? a.s : 1u;  // a bin passes with at least max(s, 1) l-mers
    constexpr int U = 4;                        // 256-bin groups per wave at a time
    const int64_t n4 = a.nb / 4;
    const int64_t per = ((a.nwb + a.parts - 1) / a.parts + 4 * U - 1) / (4 * U) * (4 * U);  // words per part
    const int64_t w_lo = part * per, w_hi = std::min<int64_t>(a.nwb, w_lo + per);
    uint32_t ne = 0, ms = 0;  // ne counts whole ballots (the same in every lane); a trial has fewer than 2^32 windows
    for (int64_t g0 = w_lo / 4 + (int64_t)wv * U; 4 * g0 < w_hi; g0 += 4 * U) {
        uint4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = (g0 + u) * 64 + lane;  // 16-byte load index
            v[u] = 4 * (g0 + u) < w_hi && i < n4 ? cnt[i] : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t c[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
            uint64_t bal[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool p = c[q] >= smin;
                bal[q] = __ballot(p);
                ne += (uint32_t)__popcll(bal[q]);
                ms += p ? c[q] : 0u;
            }
            const int64_t wi = 4 * (g0 + u) + lane;
            if (lane < 4 && wi < w_hi) {
                const int sh = 16 * lane;
                bits[wi] = ((bal[0] >> sh) & 0xffffull) | (((bal[1] >> sh) & 0xffffull) << 16) |
                           (((bal[2] >> sh) & 0xffffull) << 32) | (((bal[3] >> sh) & 0xffffull) << 48);
            }
        }
    }
    const uint32_t mst = wave_sum(ms);
    __shared__ uint64_t red[2][4];
    if (lane == 0) {
        red[0][wv] = ne;
        red[1][wv] = mst;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int64_t tb = (int64_t)(red[0][0] + red[0][1] + red[0][2] + red[0][3]);
        const int64_t tm = (int64_t)(red[1][0] + red[1][1] + red[1][2] + red[1][3]);
        if (a.parts > 1) {
            a.ws.nep[(int64_t)j * a.parts + part] = tb;
            a.ws.msp[(int64_t)j * a.parts + part] = tm;
        } else {
            a.ws.ne[j] = tb;
            a.ws.ms[j] = tm;
        }
    }
}

// bit i of a 16-bit value moved to bit 4i
__device__ __forceinline__ uint64_t spread4(uint64_t x)
{
    uint64_t v = x & 0xffffull;
    v = (v | (v << 24)) & 0x000000ff000000ffull;
    v = (v | (v << 12)) & 0x000f000f000f000full;
    v = (v | (v << 6)) & 0x0303030303030303ull;
    v = (v | (v << 3)) & 0x1111111111111111ull;
    return v;
}

// a bitmap word from lane-major order (bit 16q + i: key 4i + q) to key order
__device__ __forceinline__ uint64_t word_in_key_order(uint64_t b)
{
    return spread4(b) | (spread4(b >> 16) << 1) | (spread4(b >> 32) << 2) | (spread4(b >> 48) << 3);
}

// exclusive scan of per-trial (or per trial-slice) totals, one workgroup:
// bases of every entry, the required totals in n_out, capacity status, and
// on request the list of heavy entries
__global__ void __launch_bounds__(1024) k_tot_scan(const TotScan a)
{
    __shared__ int64_t sa[1024], sb[1024];
    __shared__ int64_t carry[3];
    __shared__ unsigned long long hmax;
    __shared__ uint32_t hw[16];
    const int wave = threadIdx.x >> 6, lane = lane_id();
    if (threadIdx.x == 0) {
        carry[0] = carry[1] = carry[2] = 0;
        hmax = 0;
    }
    __syncthreads();
    for (int64_t base = 0; base < a.n; base += 1024) {
        const int64_t j = base + threadIdx.x;
        int64_t ve = 0, vm = 0;
        if (j < a.n) {
            if (a.parts > 1) {
                for (int q = 0; q < a.parts; ++q) {
                    ve += a.ne[j * a.parts + q];
                    vm += a.ms[j * a.parts + q];
                }
                a.ne_sum[j] = ve;
                a.ms_sum[j] = vm;
            } else {
                ve = a.ne[j];
                vm = a.ms[j];
            }
        }
        sa[threadIdx.x] = ve;
        sb[threadIdx.x] = vm;
        const bool h = a.heavy && j < a.n && ve > a.heavy_above;
        if (h) atomicMax(&hmax, (unsigned long long)ve);
        const uint64_t hb = __ballot(h);
        if (lane == 0) hw[wave] = (uint32_t)__popcll(hb);
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
        if (h) {
            int64_t at = carry[2] + __popcll(hb & lanemask_lt());
            for (int w = 0; w < wave; ++w) at += hw[w];
            a.heavy[at] = (int32_t)j;
        }
        __syncthreads();
        if (threadIdx.x == 1023) {
            carry[0] += sa[1023];
            carry[1] += sb[1023];
            int64_t nh = 0;
            for (int w = 0; w < 16; ++w) nh += hw[w];
            carry[2] += nh;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.n_out[0] = carry[0];
        a.n_out[1] = carry[1];
        if ((carry[0] > a.cap_b || carry[1] > a.cap_m) && a.status) atomicOr(a.status, PM_STATUS_CAPACITY);
        if (a.heavy) a.n_heavy[0] = carry[2];
        if (a.max_heavy) a.max_heavy[0] = (int64_t)hmax;
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

// ---------------------------------------------------------------- members
constexpr int kSelU = 8;                   // window loads in flight per lane
constexpr int kSelChunk = 4 * 64 * kSelU;  // windows per workgroup step
constexpr int kSelBitsMin = 6;             // flagged lanes from which a wave groups by key bits
constexpr uint32_t kNoSlot = 0xffffffffu;
constexpr int kSelListCap = 256;           // passing windows each wave may list in a trial of few members

struct Group {
    int head;       // lowest lane holding the same key
    uint32_t rank;  // lanes below this one holding the same key
    uint32_t n;     // lanes holding the key (set at the head)
};

// Groups the flagged lanes of a wave by key (keys below 2^nbits).  With few
// flagged lanes, one ballot per distinct key; with many, each lane's peers
// (the flagged lanes holding its key) as the AND, over the nbits bits of the
// key, of the lanes that agree with it on that bit: VALU and scalar work only,
// where a sort across the wave was a chain of dependent cross-lane moves.
// Both give the same answer.
__device__ __forceinline__ Group group_by_key(bool flag, uint32_t key, int nbits)
{
    const int lane = lane_id();
    const uint64_t bal = __ballot(flag);
    Group g{lane, 0u, 0u};
    if (__popcll(bal) < kSelBitsMin) {
        uint64_t left = bal;
        while (left) {
            const int leader = __ffsll((unsigned long long)left) - 1;
            const uint32_t lk = __shfl(key, leader);
            const uint64_t peers = __ballot(flag && key == lk);
            if ((peers >> lane) & 1ull) {
                g.head = leader;
                g.rank = (uint32_t)__popcll(peers & lanemask_lt());
                g.n = (uint32_t)__popcll(peers);
            }
            left &= ~peers;
        }
        return g;
    }
    uint64_t peers = bal;
    for (int b = 0; b < nbits; ++b) {
        const bool bit = (key >> b) & 1u;
        const uint64_t on = __ballot(bit);
        peers &= bit ? on : ~on;
    }
    if (flag) {
        g.head = __ffsll((unsigned long long)peers) - 1;
        g.rank = (uint32_t)__popcll(peers & lanemask_lt());
        g.n = (uint32_t)__popcll(peers);
    }
    return g;
}

// bucket number of a passing key within its trial
__device__ __forceinline__ uint32_t local_bucket(const uint64_t *bm, const uint32_t *wcnt, uint32_t key)
{
    const uint32_t wd = key >> 6;
    return wcnt[wd] + (uint32_t)__popcll(bm[wd] & ((1ull << (key & 63u)) - 1ull));
}

// Bucket records and member lists of trial j, which has ne > 0 passing keys,
// for its buckets r0 .. r0 + cb - 1 (all of them when ne <= cb), by one
// workgroup of four waves.  Member cursors: rows[q][bucket - r0] in LDS.  A
// trial with more buckets than cb is taken by several workgroups, one range
// of buckets each, every one of them reading all of the trial's windows.
__device__ void emit_trial(const SelArgs &a, int j, int64_t ne, int64_t r0, uint64_t *bm, uint32_t *tmp)
{
    uint32_t *wcnt = reinterpret_cast<uint32_t *>(bm + a.nwb);  // [nwb] -> buckets before the word
    uint32_t *wsz = wcnt + a.nwb;                               // [nwb] -> members before the word
    uint32_t *rows = wsz + a.nwb;                               // [4][cb]
    const int tid = threadIdx.x, wv = tid >> 6, lane = lane_id();
    const int cb = a.cb;
    const bool whole = r0 == 0 && ne <= cb;                           // one range: every bucket
    const uint32_t nr = (uint32_t)std::min<int64_t>(cb, ne - r0);     // the range's buckets
    const uint32_t rlo = (uint32_t)r0, rhi = rlo + nr;
    const uint32_t *cnt = a.counts + (int64_t)j * a.nb;
    const uint64_t *bits = a.ws.bits + (int64_t)j * a.nwb;
    const int64_t bbase = a.ws.bb[j], mbase = a.ws.mb[j];
    const pm_inst I = a.inst ? a.inst[a.item_inst[j]] : a.one;

    // ---- the bitmap, and per word the total size of its passing buckets: a
    // wave takes four groups of 64 words at once (one load each) and gathers
    // the counts of eight non-empty words at a time
    for (int base = wv * 64; base < a.nwb; base += 4 * 256) {
        uint64_t b[4];
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int wi = base + 256 * it + lane;
            b[it] = wi < a.nwb ? bits[wi] : 0ull;
        }
#pragma unroll
        for (int it = 0; it < 4; ++it)
            if (__ballot(b[it] != 0ull)) b[it] = word_in_key_order(b[it]);
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int w0 = base + 256 * it, wi = w0 + lane;
            uint32_t sz = 0;
            uint64_t nz = __ballot(b[it] != 0ull);
            while (nz) {
                constexpr int G = 8;
                int idx[G];
                uint32_t c[G];
#pragma unroll
                for (int u = 0; u < G; ++u) {
                    idx[u] = nz ? __ffsll((unsigned long long)nz) - 1 : -1;
                    nz &= nz - 1ull;
                }
#pragma unroll
                for (int u = 0; u < G; ++u) {
                    c[u] = 0u;
                    if (idx[u] >= 0) {
                        const uint32_t lo = __shfl((uint32_t)b[it], idx[u]);
                        const uint32_t hi = __shfl((uint32_t)(b[it] >> 32), idx[u]);
                        if (((((uint64_t)hi << 32) | lo) >> lane) & 1ull)
                            c[u] = cnt[(int64_t)(w0 + idx[u]) * 64 + lane];
                    }
                }
#pragma unroll
                for (int u = 0; u < G; ++u)
                    if (idx[u] >= 0) {
                        const uint32_t t = wave_sum(c[u]);
                        if (lane == idx[u]) sz = t;
                    }
            }
            if (wi < a.nwb) {
                bm[wi] = b[it];
                wcnt[wi] = (uint32_t)__popcll(b[it]);
                wsz[wi] = sz;
            }
        }
    }
    __syncthreads();
    block_excl_scan(wcnt, a.nwb, tmp);
    block_excl_scan(wsz, a.nwb, tmp);

    // ---- bucket records in key order (a word's buckets are its set lanes),
    // and every bucket's cursor row: its first slot, then zeros; the counts of
    // eight non-empty words with buckets in the range are read at a time
    for (int w0 = wv * 64; w0 < a.nwb; w0 += 256) {
        const int wi = w0 + lane;
        uint64_t nz = __ballot(wi < a.nwb && bm[wi] != 0ull && wcnt[wi] < rhi &&
                               wcnt[wi] + (uint32_t)__popcll(bm[wi]) > rlo);
        while (nz) {
            constexpr int G = 8;
            int wd[G];
            uint32_t c[G];
#pragma unroll
            for (int u = 0; u < G; ++u) {
                wd[u] = nz ? w0 + __ffsll((unsigned long long)nz) - 1 : -1;
                nz &= nz - 1ull;
            }
#pragma unroll
            for (int u = 0; u < G; ++u) {
                c[u] = 0u;
                if (wd[u] >= 0 && ((bm[wd[u]] >> lane) & 1ull)) c[u] = cnt[(uint32_t)wd[u] * 64u + (uint32_t)lane];
            }
#pragma unroll
            for (int u = 0; u < G; ++u) {
                if (wd[u] < 0) continue;
                const int w = wd[u];
                const uint64_t wb = bm[w];
                const bool set = (wb >> lane) & 1ull;
                const uint32_t key = (uint32_t)w * 64u + (uint32_t)lane;
                const uint32_t frel = wsz[w] + wave_incl_scan(c[u]) - c[u];  // first slot within the trial
                const uint32_t bi = wcnt[w] + (uint32_t)__popcll(wb & lanemask_lt());
                const int64_t b = bbase + bi;
                if (set && bi >= rlo && bi < rhi) {
                    if (b < a.cap_b) a.buckets[b] = pm_bucket{(uint32_t)j, key, c[u], (uint32_t)(mbase + frel)};
                    const uint32_t ri = bi - rlo;
                    rows[ri] = frel;
                    rows[cb + ri] = rows[2 * cb + ri] = rows[3 * cb + ri] = 0u;
                }
            }
        }
    }
    __syncthreads();

    const uint32_t *kj = a.keys + I.key_base + (int64_t)(j - I.first_item) * I.x;
    const int64_t x = I.x;
    const int64_t nb = a.nb;
    // the bitmap as 32-bit words (little-endian halves of the 64-bit ones)
    const uint32_t *bm32 = reinterpret_cast<const uint32_t *>(bm);
    const uint32_t nb32 = (uint32_t)nb;
    const int nbits = 32 - __builtin_clz(nb32 - 1u);  // key bits (|Sigma|^k >= 4)
    auto passing = [&](uint32_t key) { return key < nb32 && ((bm32[key >> 5] >> (key & 31u)) & 1u); };

    if (whole && a.ws.ms[j] <= 4 * kSelListCap) {
        // few members: each wave lists the passing windows of its quarter of
        // the trial in order (no barrier), then one wave places the four lists,
        // which together are in window order, with the buckets' cursors (row 0)
        uint32_t *lw = rows + cb;                // [4][cap] windows
        uint32_t *lk = lw + 4 * kSelListCap;     // [4][cap] their keys
        const int64_t lo = x * wv / 4, hi = x * (wv + 1) / 4;
        uint32_t n = 0;
        uint32_t nk[kSelU];
#pragma unroll
        for (int u = 0; u < kSelU; ++u) {
            const int64_t w = lo + 64 * u + lane;
            nk[u] = w < hi ? kj[w] : 0u;
        }
        for (int64_t wb = lo; wb < hi; wb += 64 * kSelU) {
            uint32_t kk[kSelU];
#pragma unroll
            for (int u = 0; u < kSelU; ++u) kk[u] = nk[u];
            if (wb + 64 * kSelU < hi) {
#pragma unroll
                for (int u = 0; u < kSelU; ++u) {
                    const int64_t w = wb + 64 * kSelU + 64 * u + lane;
                    nk[u] = w < hi ? kj[w] : 0u;
                }
            }
#pragma unroll
            for (int u = 0; u < kSelU; ++u) {
                const int64_t w = wb + 64 * u + lane;
                const bool f = w < hi && passing(kk[u]);
                const uint64_t bal = __ballot(f);
                if (bal == 0ull) continue;
                const uint32_t pos = n + (uint32_t)__popcll(bal & lanemask_lt());
                if (f && pos < (uint32_t)kSelListCap) {
                    lw[wv * kSelListCap + pos] = (uint32_t)w;
                    lk[wv * kSelListCap + pos] = kk[u];
                }
                n += (uint32_t)__popcll(bal);
            }
        }
        if (lane == 0) tmp[wv] = n;
        __syncthreads();
        const uint32_t n0 = tmp[0], n1 = tmp[1], n2 = tmp[2], n3 = tmp[3];
        const uint32_t cap = (uint32_t)kSelListCap;
        if (n0 <= cap && n1 <= cap && n2 <= cap && n3 <= cap) {
            if (wv == 0) {
                const uint32_t e1 = n0, e2 = e1 + n1, e3 = e2 + n2, total = e3 + n3;
                for (uint32_t e0 = 0; e0 < total; e0 += 64) {
                    const uint32_t e = e0 + (uint32_t)lane;
                    const bool valid = e < total;
                    const uint32_t q = (e >= e1) + (e >= e2) + (e >= e3);
                    const uint32_t at = q * cap + e - (q == 0 ? 0u : q == 1 ? e1 : q == 2 ? e2 : e3);
                    const uint32_t w = valid ? lw[at] : 0u, key = valid ? lk[at] : 0u;
                    const Group g = group_by_key(valid, key, nbits);
                    uint32_t old = kNoSlot;
                    if (valid && g.head == lane) {
                        const uint32_t bi = local_bucket(bm, wcnt, key);
                        if (bbase + bi < a.cap_b) {
                            old = rows[bi];
                            rows[bi] = old + g.n;
                        }
                    }
                    old = __shfl(old, g.head);
                    if (valid && old != kNoSlot) {
                        const int64_t slot = mbase + old + g.rank;
                        if (slot < a.cap_m) a.members[slot] = w;
                    }
                }
            }
            return;
        }
        // a quarter held more than its list: the chunked placement below, with
        // rows 1-3 (which the lists overwrote) cleared again
        for (int64_t bi = tid; bi < ne; bi += 256) rows[cb + bi] = rows[2 * cb + bi] = rows[3 * cb + bi] = 0u;
        __syncthreads();
    }
    if (!whole || ne > kSelChunk / 2) {
        // more buckets than half a chunk's windows (two sweeps over them per
        // chunk would cost more than the chunk), or a range of a trial with
        // more buckets than the LDS rows hold: the windows go by quarters
        // (wave q owns the q-th quarter) in two passes: waves 0-2 count the
        // members of the range's buckets into rows 1-3 with LDS atomics, one
        // sweep turns rows 0-3 into each wave's first slot, and every wave
        // places its quarter's members of the range
        const uint32_t lo = (uint32_t)(x * wv / 4), hi = (uint32_t)(x * (wv + 1) / 4);  // x < 2^32
        if (wv < 3) {
            for (uint32_t wb = lo; wb < hi; wb += 64 * kSelU) {
                uint32_t kk[kSelU];
#pragma unroll
                for (int u = 0; u < kSelU; ++u) {
                    const uint32_t w = wb + 64 * u + lane;
                    kk[u] = w < hi ? kj[w] : 0u;
                }
#pragma unroll
                for (int u = 0; u < kSelU; ++u)
                    if (wb + 64 * u + lane < hi && passing(kk[u])) {
                        const uint32_t ri = local_bucket(bm, wcnt, kk[u]) - rlo;
                        if (ri < nr) atomicAdd(rows + (wv + 1) * cb + ri, 1u);
                    }
            }
        }
        __syncthreads();
        for (uint32_t ri = tid; ri < nr; ri += 256) {
            const uint32_t r1 = rows[ri] + rows[cb + ri];
            const uint32_t r2 = r1 + rows[2 * cb + ri];
            rows[cb + ri] = r1;
            rows[2 * cb + ri] = r2;
            rows[3 * cb + ri] += r2;
        }
        __syncthreads();
        for (uint32_t wb = lo; wb < hi; wb += 64 * kSelU) {
            uint32_t kk[kSelU], ri[kSelU];
            uint64_t peers[kSelU];
#pragma unroll
            for (int u = 0; u < kSelU; ++u) {
                const uint32_t w = wb + 64 * u + lane;
                kk[u] = w < hi ? kj[w] : 0u;
            }
            uint32_t nflag = 0;
#pragma unroll
            for (int u = 0; u < kSelU; ++u) {
                const uint32_t w = wb + 64 * u + lane;
                ri[u] = 0xffffffffu;
                if (w < hi && passing(kk[u])) ri[u] = local_bucket(bm, wcnt, kk[u]) - rlo;
                peers[u] = __ballot(ri[u] < nr);
                nflag += (uint32_t)__popcll(peers[u]);
            }
            if (nflag >= (uint32_t)(kSelBitsMin * kSelU)) {
                // many members: the groups of all kSelU steps at once (their
                // ballots over the key bits interleave), then one returning LDS
                // atomic per group head, in step order (a wave's LDS operations
                // complete in order, so a bucket's cursor advances step by step)
                for (int b = 0; b < nbits; ++b)
#pragma unroll
                    for (int u = 0; u < kSelU; ++u) {
                        const bool bit = (kk[u] >> b) & 1u;
                        const uint64_t on = __ballot(bit);
                        peers[u] &= bit ? on : ~on;
                    }
                uint32_t old[kSelU];
                int head[kSelU];
#pragma unroll
                for (int u = 0; u < kSelU; ++u) {
                    const bool f = ri[u] < nr;
                    head[u] = f ? __ffsll((unsigned long long)peers[u]) - 1 : lane;
                    old[u] = kNoSlot;
                    if (f && head[u] == lane && bbase + rlo + ri[u] < a.cap_b)
                        old[u] = atomicAdd(rows + wv * cb + ri[u], (uint32_t)__popcll(peers[u]));
                }
#pragma unroll
                for (int u = 0; u < kSelU; ++u) {
                    const uint32_t o = __shfl(old[u], head[u]);
                    if (ri[u] < nr && o != kNoSlot) {
                        const int64_t slot = mbase + o + (uint32_t)__popcll(peers[u] & lanemask_lt());
                        if (slot < a.cap_m) a.members[slot] = wb + 64 * u + lane;
                    }
                }
                continue;
            }
#pragma unroll
            for (int u = 0; u < kSelU; ++u) {
                const uint32_t w = wb + 64 * u + lane;
                const bool f = ri[u] < nr;
                if (peers[u] == 0ull) continue;
                const Group g = group_by_key(f, kk[u], nbits);
                uint32_t old = kNoSlot;
                if (f && g.head == lane && bbase + rlo + ri[u] < a.cap_b) {
                    uint32_t *r = rows + wv * cb + ri[u];
                    old = *r;
                    *r = old + g.n;
                }
                old = __shfl(old, g.head);
                if (f && old != kNoSlot) {
                    const int64_t slot = mbase + old + g.rank;
                    if (slot < a.cap_m) a.members[slot] = w;
                }
            }
        }
        return;
    }
    {
        // chunks of 2048 windows, wave q owning the q-th quarter of each: rows
        // 1-3 count the members of waves 0-2 per bucket, a sweep turns rows
        // 0-3 into each wave's first slot, the waves place their members, and
        // wave 3's row, now the first free slot, becomes row 0 again
        // the next chunk's keys are loaded while this one is placed
        uint32_t nk[kSelU];
#pragma unroll
        for (int u = 0; u < kSelU; ++u) {
            const int64_t w = (int64_t)wv * 64 * kSelU + 64 * u + lane;
            nk[u] = w < x ? kj[w] : 0u;
        }
        for (int64_t c0 = 0; c0 < x; c0 += kSelChunk) {
            const int64_t wb = c0 + (int64_t)wv * 64 * kSelU;
            uint32_t kk[kSelU];
#pragma unroll
            for (int u = 0; u < kSelU; ++u) kk[u] = nk[u];
            if (c0 + kSelChunk < x) {
#pragma unroll
                for (int u = 0; u < kSelU; ++u) {
                    const int64_t w = wb + kSelChunk + 64 * u + lane;
                    nk[u] = w < x ? kj[w] : 0u;
                }
            }
            uint32_t fl = 0;  // bit u: this lane's window of step u passes
            if (c0 + kSelChunk <= x) {
#pragma unroll
                for (int u = 0; u < kSelU; ++u) fl |= passing(kk[u]) ? 1u << u : 0u;
            } else {
                const int left = (int)(x - wb);  // windows of this wave in the last chunk
#pragma unroll
                for (int u = 0; u < kSelU; ++u) fl |= 64 * u + lane < left && passing(kk[u]) ? 1u << u : 0u;
            }
            if (!__syncthreads_or(fl != 0u)) continue;
            if (wv < 3) {
                // counts only: one LDS atomic per member, no grouping
#pragma unroll
                for (int u = 0; u < kSelU; ++u)
                    if ((fl >> u) & 1u) atomicAdd(rows + (wv + 1) * cb + local_bucket(bm, wcnt, kk[u]), 1u);
            }
            __syncthreads();
            for (int64_t bi = tid; bi < ne; bi += 256) {
                const uint32_t r1 = rows[bi] + rows[cb + bi];
                const uint32_t r2 = r1 + rows[2 * cb + bi];
                rows[cb + bi] = r1;
                rows[2 * cb + bi] = r2;
                rows[3 * cb + bi] += r2;
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kSelU; ++u) {
                const bool f = (fl >> u) & 1u;
                if (__ballot(f) == 0ull) continue;
                const Group g = group_by_key(f, kk[u], nbits);
                uint32_t old = kNoSlot;
                if (f && g.head == lane) {
                    const uint32_t bi = local_bucket(bm, wcnt, kk[u]);
                    if (bbase + bi < a.cap_b) {
                        uint32_t *r = rows + wv * cb + bi;
                        old = *r;
                        *r = old + g.n;
                    }
                }
                old = __shfl(old, g.head);
                if (f && old != kNoSlot) {
                    const int64_t slot = mbase + old + g.rank;
                    if (slot < a.cap_m) a.members[slot] = (uint32_t)(wb + 64 * u + lane);
                }
            }
            __syncthreads();
            for (int64_t bi = tid; bi < ne; bi += 256) {
                rows[bi] = rows[3 * cb + bi];
                rows[cb + bi] = rows[2 * cb + bi] = rows[3 * cb + bi] = 0u;
            }
            __syncthreads();
        }
        return;
    }
}

// one workgroup per trial whose buckets fit the LDS rows
__global__ void __launch_bounds__(256) k_sel_emit(const SelArgs a)
{
    extern __shared__ __align__(16) uint64_t bm[];
    __shared__ uint32_t tmp[256];
    const int j = blockIdx.x;
    if (j == 0 && threadIdx.x < 3) a.ws.qctr[threadIdx.x] = 0;  // the heavy launches' queues, for after this one
    const int64_t ne = a.ws.ne[j];
    if (ne <= a.take_lo || ne > a.take_hi) return;
    emit_trial(a, j, ne, 0, bm, tmp);
}

// the trials with more buckets than that, listed by the scan; a fixed grid
// of workgroups takes the (range of cb buckets, trial) units of the trials in
// the launch's range of bucket counts from a work queue (trials differ in
// size by an order of magnitude), range-major (so that the trials' first
// ranges, which every trial has, come first)
__global__ void __launch_bounds__(256) k_sel_emit_heavy(const SelArgs a)
{
    extern __shared__ __align__(16) uint64_t bm[];
    __shared__ uint32_t tmp[256];
    __shared__ int64_t claim;
    // bucket ranges of the largest heavy trial (at most a.ranges)
    const int64_t rg = std::min<int64_t>(a.ranges, (a.ws.qctr[3] + a.cb - 1) / a.cb);
    const int64_t nh = *a.ws.n_heavy, nu = nh * rg;
    if (nu == 0) return;  // no heavy trial: no queue traffic
    unsigned long long *q = reinterpret_cast<unsigned long long *>(a.ws.qctr + a.tier);
    for (;;) {
        if (threadIdx.x == 0) claim = (int64_t)atomicAdd(q, 1ull);
        __syncthreads();
        const int64_t un = claim;
        __syncthreads();
        if (un >= nu) break;  // every workgroup ends here once the queue is past its end
        const int j = a.ws.heavy[un % nh];
        const int64_t ne = a.ws.ne[j], r0 = (un / nh) * (int64_t)a.cb;  // range-major
        if (ne <= a.take_lo || ne > a.take_hi || r0 >= ne) continue;  // uniform over the workgroup
        emit_trial(a, j, ne, r0, bm, tmp);
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

// SW lanes per bucket (16 for l <= 16, else 32; 64 / SW buckets per wave);
// lane j of a bucket's group owns column j
template <int SW>
__global__ void __launch_bounds__(256) k_profile(const ProfArgs a)
{
    constexpr int NB = 64 / SW;  // buckets per wave
    __shared__ uint32_t cnt[4][NB][20 * SW];
    const int wv = threadIdx.x >> 6, lane = lane_id(), sub = lane / SW, j = lane % SW;
    const int64_t b = ((int64_t)blockIdx.x * 4 + wv) * NB + sub;
    int64_t nvalid = a.n_dev ? *a.n_dev : a.B;
    if (nvalid > a.B) nvalid = a.B;
    if (((int64_t)blockIdx.x * 4 + wv) * NB >= nvalid) return;  // the wave's first bucket (uniform)
    const bool live = b < nvalid;
    uint32_t *C = cnt[wv][sub];
    for (int i = j; i < a.A * SW; i += SW) C[i] = 0;
    pm_bucket bk{0u, 0u, 0u, 0u};
    if (live) bk = a.buckets[b];
    const pm_inst I = a.inst ? a.inst[a.item_inst[live ? bk.trial : 0]] : a.one;
    const int64_t lm1 = a.l - 1;
    const uint32_t size = live && (int64_t)bk.first + bk.size <= a.cap_m ? bk.size : 0u;
    // SW members at a time: lane j finds where member j starts, then every
    // column lane reads the members' symbols one after another
    uint32_t most = size;  // the wave's largest bucket
#pragma unroll
    for (int o = SW; o < 64; o <<= 1) {
        const uint32_t t = __shfl_xor(most, o);
        most = t > most ? t : most;
    }
    for (uint32_t r0 = 0; r0 < most; r0 += SW) {
        const uint32_t nr = size > r0 ? (size - r0 < (uint32_t)SW ? size - r0 : (uint32_t)SW) : 0u;
        int64_t Pm = 0;
        if ((uint32_t)j < nr) {
            const int64_t w = a.members[(int64_t)bk.first + r0 + j];
            int lo = 0, hi = I.t;  // last sequence whose first window <= w
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (I.offsets[mid] - (int64_t)mid * lm1 <= w) lo = mid;
                else hi = mid;
            }
            Pm = w + (int64_t)lo * lm1;
        }
        const uint32_t nmost = most - r0 < (uint32_t)SW ? most - r0 : (uint32_t)SW;
        for (uint32_t r = 0; r < nmost; ++r) {
            const int64_t P = __shfl(Pm, sub * SW + (int)r);
            if (r < nr && j < a.l) {
                const uint32_t code = a.A == 4 ? dna_sym(I.packed, P + j) : prot_sym(I.packed, P + j);
                C[code * SW + j] += 1;
            }
        }
    }
    if (!live) return;
    uint32_t *out = a.profile + b * a.A * a.l;
    for (int c = 0; c < a.A; ++c)
        if (j < a.l) out[c * a.l + j] = C[c * SW + j];
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

// |Sigma|^k for the count-table selection, or -1 above 2^19 bins
static int64_t sel_bins(int A, int k)
{
    if ((A != 4 && A != 20) || k < 1) return -1;
    int64_t nb = 1;
    for (int i = 0; i < k; ++i) {
        nb *= A;
        if (nb > (1ll << 19)) return -1;
    }
    return nb;
}

extern "C" size_t pm_select_workspace(int32_t alphabet, int32_t k, int32_t m, int64_t cap_buckets)
{
    const int64_t nb = sel_bins(alphabet, k);
    if (nb < 0 || m < 0 || cap_buckets < 0) return 0;
    return sel_ws_bytes(m, (nb + 63) / 64);  // member cursors live in LDS: no per-bucket space
}

// dynamic LDS of the emit kernels: bitmap, word scans, cursor row 0, then
// rows 1-3 or the member lists of a trial with few members
static size_t sel_emit_lds(int64_t nwb, int64_t cb)
{
    return (size_t)(16 * nwb + 4 * cb + 4 * std::max<int64_t>(3 * cb, 8 * kSelListCap));
}

// counted: the bitmap and the per-trial totals are already in the workspace
// (projection_hash_select's hash pass wrote them), so no counting pass
static int select_launch(SelArgs &a, int64_t x_max, hipStream_t st, bool counted = false)
{
    const int64_t nwb = (a.nb + 63) / 64;
    a.nwb = (int)nwb;
    a.parts = counted ? 1 : sel_parts(a.m, nwb);
    if (!counted) {
        hipLaunchKernelGGL(k_sel_count, dim3((unsigned)((int64_t)a.m * a.parts)), dim3(256), 0, st, a);
        PM_LAUNCHED();
    }
    // a trial has at most min(|Sigma|^k, x / s) passing bins; the first emit
    // launch keeps its LDS near 20 KB (eight workgroups per CU) and takes the
    // trials whose buckets fit there, a second one with all the LDS the device
    // gives takes the rest from a list the scan writes
    const int64_t ne_bound = std::min<int64_t>(a.nb, x_max / std::max<uint32_t>(a.s, 1u));
    const int64_t lds_max = device_lds_bytes() - 2048;  // the emit kernels hold 1 KB of static LDS
    const int64_t fit = (lds_max - 16 * nwb) / 16;
    const int64_t cb_a = std::max<int64_t>(1, std::min<int64_t>(ne_bound, std::max<int64_t>(256, (20480 - 16 * nwb) / 16)));
    const bool heavy = a.nb > cb_a;  // counts not written by projection_hash may pass anywhere
    TotScan ts{a.ws.ne, a.ws.ms, a.ws.bb, a.ws.mb, a.m, a.cap_b, a.cap_m, a.n_out, a.status};
    if (a.parts > 1) {
        ts.ne = a.ws.nep;
        ts.ms = a.ws.msp;
        ts.parts = a.parts;
        ts.ne_sum = a.ws.ne;
        ts.ms_sum = a.ws.ms;
    }
    if (heavy) {
        ts.heavy = a.ws.heavy;
        ts.n_heavy = a.ws.n_heavy;
        ts.heavy_above = cb_a;
        ts.max_heavy = a.ws.qctr + 3;
    }
    if (int rc = launch_tot_scan(ts, st)) return rc;
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)k_sel_emit, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_max);
        (void)hipFuncSetAttribute((const void *)k_sel_emit_heavy, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds_max);
        (void)hipGetLastError();  // an unsupported attribute must not poison the launch check
        attr = true;
    }
    a.take_lo = 0;
    a.take_hi = cb_a;
    a.cb = (int)cb_a;
    hipLaunchKernelGGL(k_sel_emit, dim3(a.m), dim3(256), sel_emit_lds(nwb, cb_a), st, a);
    PM_LAUNCHED();
    if (heavy) {
        // the heavy trials in tiers of LDS rows sized for four, two and one
        // workgroups per CU (the fewer rows, the more workgroups hide each
        // other's latency); the last tier also takes the trials beyond every
        // LDS row count, as several ranges of buckets
        int64_t lo = cb_a;
        int tier = 0;
        for (const int per_cu : {4, 2, 1}) {
            int64_t cb = (lds_max / per_cu - 2048 - 16 * nwb) / 16;  // 1 KB static LDS, 1 KB headroom
            if (per_cu == 1) cb = std::max<int64_t>(lo, std::min<int64_t>(ne_bound, fit));
            else if (cb <= lo) continue;
            cb = std::min<int64_t>(cb, std::max<int64_t>(lo, ne_bound));
            a.cb = (int)cb;
            a.take_lo = lo;
            a.take_hi = per_cu == 1 ? INT64_MAX : cb;
            // only the last tier has trials with more buckets than its rows
            a.ranges = per_cu == 1 ? (int)((std::max<int64_t>(ne_bound, cb) + cb - 1) / cb) : 1;
            a.tier = tier++;
            const int grid = std::min<int32_t>(a.m, 1024);
            hipLaunchKernelGGL(k_sel_emit_heavy, dim3(grid), dim3(256), sel_emit_lds(nwb, cb), st, a);
            PM_LAUNCHED();
            lo = cb;
            if (lo >= ne_bound) break;  // no trial has more buckets
        }
    }
    return PM_OK;
}

static int check_select_args(int A, int k, int32_t items, const uint32_t *keys, const uint32_t *counts,
                             const int64_t *n_out, void *ws, size_t ws_bytes, pm_bucket *buckets,
                             int64_t cap_buckets, uint32_t *members, int64_t cap_members)
{
    if (items < 1) return fail(PM_EINVAL, "m must be >= 1");
    if (sel_bins(A, k) < 0) return fail(PM_ERANGE, "|Sigma|^k above 2^19");
    if (!keys || !counts || !n_out || !ws) return fail(PM_EINVAL, "keys, counts, n_out and ws are required");
    if (cap_buckets < 0 || cap_members < 0) return fail(PM_EINVAL, "negative capacity");
    if ((cap_buckets > 0 && !buckets) || (cap_members > 0 && !members))
        return fail(PM_EINVAL, "NULL output with a non-zero capacity");
    if (cap_members > 0xffffffffll) return fail(PM_ERANGE, "cap_members must be below 2^32");
    if (ws_bytes < pm_select_workspace(A, k, items, cap_buckets)) return fail(PM_EINVAL, "workspace too small");
    if (reinterpret_cast<uintptr_t>(ws) & 7) return fail(PM_EINVAL, "workspace must be 8-byte aligned");
    return PM_OK;
}

namespace pm {

int check_select_ws(int A, int k, int32_t items, const uint32_t *keys, const uint32_t *counts,
                    const int64_t *n_out, void *ws, size_t ws_bytes, pm_bucket *buckets, int64_t cap_buckets,
                    uint32_t *members, int64_t cap_members)
{
    return check_select_args(A, k, items, keys, counts, n_out, ws, ws_bytes, buckets, cap_buckets, members,
                             cap_members);
}

__global__ void k_sel_zero(int64_t *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

int select_counted_prepare(void *ws, int32_t m, int A, int k, SelCounted *out, hipStream_t st)
{
    const int64_t nb = sel_bins(A, k), nwb = (nb + 63) / 64;
    const SelWs w = carve(ws, m, nwb);
    // ne and ms are adjacent: [m] each
    hipLaunchKernelGGL(k_sel_zero, dim3((unsigned)((2 * (int64_t)m + 255) / 256)), dim3(256), 0, st, w.ne,
                       2 * (int64_t)m);
    PM_LAUNCHED();
    *out = SelCounted{w.bits, w.ne, w.ms, nwb};
    return PM_OK;
}

int select_counted(const pm_inst &one, const pm_inst *inst, const int32_t *item_inst, int A, int k,
                   const uint32_t *keys, const uint32_t *counts, int32_t m, uint32_t s, pm_bucket *buckets,
                   int64_t cap_buckets, uint32_t *members, int64_t cap_members, int64_t *n_out, void *ws,
                   uint32_t *status, int64_t x_max, hipStream_t st)
{
    SelArgs a{};
    a.one = one;
    a.inst = inst;
    a.item_inst = item_inst;
    a.keys = keys;
    a.counts = counts;
    a.buckets = buckets;
    a.members = members;
    a.n_out = n_out;
    a.status = status;
    a.nb = sel_bins(A, k);
    a.ws = carve(ws, m, (a.nb + 63) / 64);
    a.cap_b = cap_buckets;
    a.cap_m = cap_members;
    a.m = m;
    a.s = s;
    return select_launch(a, x_max, st, true);
}

}  // namespace pm

extern "C" int bucket_select(const pm_seqs *S, int32_t l, int32_t k, const uint32_t *keys,
                             const uint32_t *counts, int32_t m, uint32_t s, pm_bucket *buckets,
                             int64_t cap_buckets, uint32_t *members, int64_t cap_members,
                             int64_t *n_out, void *ws, size_t ws_bytes, uint32_t *status, void *stream)
{
    clear_error();
    int rc = check_seqs(S, l);
    if (rc) return rc;
    if (k < 1 || k > l) return fail(PM_EINVAL, "need 1 <= k <= l");
    if ((rc = check_select_args(S->alphabet, k, m, keys, counts, n_out, ws, ws_bytes, buckets, cap_buckets, members,
                                cap_members)))
        return rc;
    SelArgs a{};
    a.one = inst_of(S, l);
    a.keys = keys;
    a.counts = counts;
    a.buckets = buckets;
    a.members = members;
    a.n_out = n_out;
    a.status = status;
    a.nb = sel_bins(S->alphabet, k);
    a.ws = carve(ws, m, (a.nb + 63) / 64);
    a.cap_b = cap_buckets;
    a.cap_m = cap_members;
    a.m = m;
    a.s = s;
    return select_launch(a, a.one.x, as_stream(stream));
}

extern "C" int bucket_select_batch(const pm_batch *B, const uint32_t *keys, const uint32_t *counts, uint32_t s,
                                   pm_bucket *buckets, int64_t cap_buckets, uint32_t *members,
                                   int64_t cap_members, int64_t *n_out, void *ws, size_t ws_bytes,
                                   uint32_t *status, void *stream)
{
    clear_error();
    BatchInfo info;
    int rc = check_batch(B, &info);
    if (rc) return rc;
    if ((rc = check_select_args(B->alphabet, B->k, B->items, keys, counts, n_out, ws, ws_bytes, buckets, cap_buckets,
                                members, cap_members)))
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
    a.nb = sel_bins(B->alphabet, B->k);
    a.ws = carve(ws, B->items, (a.nb + 63) / 64);
    a.cap_b = cap_buckets;
    a.cap_m = cap_members;
    a.m = B->items;
    a.s = s;
    return select_launch(a, info.x_max, as_stream(stream));
}

static int profile_launch(const ProfArgs &a, hipStream_t st)
{
    if (a.l <= 16) {
        hipLaunchKernelGGL(k_profile<16>, dim3((unsigned)((a.B + 15) / 16)), dim3(256), 0, st, a);
    } else {
        hipLaunchKernelGGL(k_profile<32>, dim3((unsigned)((a.B + 7) / 8)), dim3(256), 0, st, a);
    }
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
