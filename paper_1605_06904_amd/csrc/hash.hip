// a1 (encode + pack) and a3/a4 (projection, keys, bucket histogram) on gfx950.
//
// Sec. 6 of the paper maps letters to integers and projects/hashes one l-mer
// per GPU thread.  Here one workgroup owns one trial (and one slice of the
// key range when the |Sigma|^k histogram does not fit in LDS): it stages the
// packed input (a few KB) in LDS, builds keys from LDS windows, writes them
// with coalesced stores and counts them in an LDS histogram of u4, u8, u16 or
// u32 counters (the width that needs the fewest key-range slices, then the
// most workgroups per CU, then the widest), then streams the histogram out as
// dense u32 counts.  A narrow counter that wraps is seen from the value its
// atomic returned (u4, u8) or from the slice's window total (u16), and such a
// slice is counted again in u32.
#include <algorithm>
#include <mutex>

#include "hash_dev.h"

namespace pm {

// ---------------------------------------------------------------- a1: pack
__device__ __forceinline__ int code_of(int A, uint32_t ch)
{
    if (ch >= 'a' && ch <= 'z') ch -= 'a' - 'A';
    if (A == 4) {
        switch (ch) {
        case 'A': return 0;
        case 'C': return 1;
        case 'T': return 2;
        case 'G': return 3;
        default: return -1;
        }
    }
    switch (ch) {
    case 'A': return 0;  case 'R': return 1;  case 'N': return 2;  case 'D': return 3;
    case 'C': return 4;  case 'Q': return 5;  case 'E': return 6;  case 'G': return 7;
    case 'H': return 8;  case 'I': return 9;  case 'L': return 10; case 'K': return 11;
    case 'M': return 12; case 'F': return 13; case 'P': return 14; case 'S': return 15;
    case 'T': return 16; case 'W': return 17; case 'Y': return 18; case 'V': return 19;
    default: return -1;
    }
}

__global__ void k_pack(int A, const uint8_t *__restrict__ ascii, int64_t n, uint32_t *__restrict__ packed,
                       int64_t nwords, uint32_t *status)
{
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nwords) return;
    const int per = A == 4 ? 16 : 6;
    const int bits = A == 4 ? 2 : 5;
    uint32_t v = 0;
    bool bad = false;
    for (int q = 0; q < per; ++q) {
        const int64_t g = w * per + q;
        int c = 0;
        if (g < n) {
            c = code_of(A, ascii[g]);
            if (c < 0) {
                bad = true;
                c = 0;
            }
        }
        v |= (uint32_t)c << (32 - bits * (q + 1));
    }
    packed[w] = v;
    if (bad && status) atomicOr(status, PM_STATUS_BAD_SYMBOL);
}

// ---------------------------------------------------------------- a3 + a4

template <bool U16>
__device__ __forceinline__ void hist_add(uint32_t *hist, uint32_t bin)
{
    if (U16) atomicAdd(hist + (bin >> 1), 1u << ((bin & 1) << 4));
    else atomicAdd(hist + bin, 1u);
}

constexpr int kHashFlagWords = 3;  // LDS words after the staged input: the slice's window total, and
                                   // its passing bins and members for projection_hash_select

// Count-table widths of k_hash.
constexpr int kHist16 = 0;       // u16 pairs: instances below 65 536 windows
constexpr int kHist16Check = 1;  // u16 pairs, slices of 65 536 windows or more counted again in u32
constexpr int kHist32 = 2;       // u32
constexpr int kHist8 = 3;        // u8 quads, a slice where a count wrapped counted again in u32
constexpr int kHist4 = 4;        // u4 octets, the same
constexpr int kHistModes = 5;

// Narrow counts hold more bins per slice, so fewer slices (each of which
// recomputes every key of its trial).  A u16 count can pass 65 535 only when
// at least 65 536 windows fall in its slice, so with kHist16Check every thread
// counts the windows of its slice (one add per window, the atomics stay
// non-returning) and a slice that received 65 536 or more is counted again in
// u32, hist_words bins per pass.  u8 counts wrap at 256 and u4 counts at 16:
// kHist8 and kHist4 increment with returning atomics and a slice where a count
// wrapped is counted again in u32 the same way (only a key with 256, or 16,
// windows or more in one trial can).
template <int A, int K, int HIST>
__global__ void __launch_bounds__(kHashThreads) k_hash(const HashArgs a)
{
    // all LDS is dynamic (the count table may take every byte the device
    // allows, so a static variable would not fit beside it)
    extern __shared__ __align__(16) uint32_t smem[];
    const int slice = blockIdx.x % a.nslices;
    const int j = blockIdx.x / a.nslices;
    const int tid = threadIdx.x;

    const uint32_t mask = a.masks[j];
    if (!mask_ok(a, mask)) {
        if (tid == 0 && slice == 0 && a.status) atomicOr(a.status, PM_STATUS_BAD_MASK);
        return;
    }

    uint32_t *hist = smem;
    uint32_t *seq = smem + a.hist_words;
    int32_t *wst = reinterpret_cast<int32_t *>(seq + a.seq_cap);  // window number of each sequence start
    uint32_t &in_slice = *reinterpret_cast<uint32_t *>(wst + a.off_cap);  // kHashFlagWords
    uint32_t *sel_acc = &in_slice + 1;                                     // [2]
    const Staged st = stage_input<A>(a, j, seq, wst);
    const pm_inst &I = st.I;
    const int64_t x = I.x;
    if (a.counts)
        for (int i = tid * 4; i < a.hist_words; i += kHashThreads * 4)
            *reinterpret_cast<uint4 *>(hist + i) = make_uint4(0, 0, 0, 0);
    if (tid == 0) in_slice = sel_acc[0] = sel_acc[1] = 0;
    __syncthreads();

    int pos[K];
    kept_positions<A, K>(mask, pos);
    const uint32_t slice_base = (uint32_t)slice * a.slice_bins;  // |Sigma|^k <= 2^24
    const int64_t kw0 = x * slice / a.nslices, kw1 = x * (slice + 1) / a.nslices;
    uint32_t *keys_j = a.keys ? a.keys + I.key_base + (int64_t)(j - I.first_item) * x : nullptr;
    uint32_t mine = 0;
    for_each_key<A, K>(a, st, pos, [&](int64_t w, uint32_t key) {
        // ordinary stores: a trial's key row is not aligned to cache lines, and
        // non-temporal stores of partial lines cost a quarter of the kernel
        if (keys_j && w >= kw0 && w < kw1) keys_j[w] = key;
        if (a.counts) {
            const uint32_t bin = key - slice_base;
            if (bin < a.slice_bins) {
                if (HIST == kHist32) {
                    atomicAdd(hist + bin, 1u);
                } else if (HIST == kHist8) {
                    const uint32_t sh = (bin & 3) << 3;
                    const uint32_t old = atomicAdd(hist + (bin >> 2), 1u << sh);
                    mine |= ((old >> sh) & 0xffu) == 0xffu;
                } else if (HIST == kHist4) {
                    const uint32_t sh = (bin & 7) << 2;
                    const uint32_t old = atomicAdd(hist + (bin >> 3), 1u << sh);
                    mine |= ((old >> sh) & 0xfu) == 0xfu;
                } else {
                    atomicAdd(hist + (bin >> 1), 1u << ((bin & 1) << 4));
                    if (HIST == kHist16Check) ++mine;
                }
            }
        }
    });
    if (!a.counts) return;
    if (HIST == kHist16Check) {
        mine = wave_sum(mine);
        if (lane_id() == 0) atomicAdd(&in_slice, mine);
    } else if (HIST == kHist8 || HIST == kHist4) {
        if (mine) in_slice = 1u << 16;  // a count wrapped: recount below
    }
    __syncthreads();

    const uint64_t left = (uint64_t)a.nb - slice_base;
    const uint32_t nvalid = left < a.slice_bins ? (uint32_t)left : a.slice_bins;  // multiple of 4
    uint32_t *out = a.counts + (int64_t)j * a.nb + slice_base;
    const int wv = tid >> 6, lane = lane_id();
    uint32_t sel_ne = 0, sel_ms = 0;  // sel_ne counts whole ballots (the same in every lane)
    // projection_hash_select: the counts v of bins base + 4 lane .. +3 (a wave
    // takes 256 bins, base a multiple of 256 from the slice's start): one
    // ballot per bin of the quad gives four bitmap words
    auto select_words = [&](uint32_t base, bool valid, const u32x4 &v) {
        uint64_t bal[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const bool p = valid && v[q] >= a.sel_smin;
            bal[q] = __ballot(p);
            sel_ne += (uint32_t)__popcll(bal[q]);
            sel_ms += p ? v[q] : 0u;
        }
        const int64_t wi = (int64_t)(slice_base + base) / 64 + lane;
        if (lane < 4 && wi < a.sel_nwb) {
            const int sh = 16 * lane;
            a.sel_bits[(int64_t)j * a.sel_nwb + wi] =
                ((bal[0] >> sh) & 0xffffull) | (((bal[1] >> sh) & 0xffffull) << 16) |
                (((bal[2] >> sh) & 0xffffull) << 32) | (((bal[3] >> sh) & 0xffffull) << 48);
        }
    };
    const bool wrapped = (HIST == kHist16Check || HIST == kHist8 || HIST == kHist4) && in_slice >= 65536u;
    if (!wrapped) {
        for (uint32_t base = 256u * wv; base < nvalid; base += kHashThreads * 4) {
            const uint32_t b4 = base + 4u * lane;
            const bool valid = b4 < nvalid;
            u32x4 v = u32x4{0u, 0u, 0u, 0u};
            if (valid) {
                if (HIST == kHist32) {
                    const uint4 w = *reinterpret_cast<const uint4 *>(hist + b4);
                    v = u32x4{w.x, w.y, w.z, w.w};
                } else if (HIST == kHist8) {
                    const uint32_t w = hist[b4 >> 2];
                    v = u32x4{w & 0xffu, (w >> 8) & 0xffu, (w >> 16) & 0xffu, w >> 24};
                } else if (HIST == kHist4) {
                    const uint32_t w = hist[b4 >> 3] >> ((b4 & 4u) << 2);
                    v = u32x4{w & 0xfu, (w >> 4) & 0xfu, (w >> 8) & 0xfu, (w >> 12) & 0xfu};
                } else {
                    const uint32_t w0 = hist[b4 >> 1], w1 = hist[(b4 >> 1) + 1];
                    v = u32x4{w0 & 0xffffu, w0 >> 16, w1 & 0xffffu, w1 >> 16};
                }
                __builtin_nontemporal_store(v, reinterpret_cast<u32x4 *>(out + b4));
            }
            if (a.sel_bits) select_words(base, valid, v);
        }
    } else {
        // a count may have wrapped: the slice counted again in u32,
        // hist_words bins per pass (a multiple of 256 with the selection)
        const uint32_t hw = (uint32_t)a.hist_words;
        for (uint32_t h0 = 0; h0 < nvalid; h0 += hw) {
            __syncthreads();
            for (int i = tid * 4; i < a.hist_words; i += kHashThreads * 4)
                *reinterpret_cast<uint4 *>(hist + i) = make_uint4(0, 0, 0, 0);
            __syncthreads();
            for_each_key<A, K>(a, st, pos, [&](int64_t, uint32_t key) {
                const uint32_t bin = key - slice_base - h0;
                if (bin < hw) atomicAdd(hist + bin, 1u);
            });
            __syncthreads();
            const uint32_t n = nvalid - h0 < hw ? nvalid - h0 : hw;
            for (uint32_t base = 256u * wv; base < n; base += kHashThreads * 4) {
                const uint32_t b4 = base + 4u * lane;
                const bool valid = b4 < n;
                u32x4 v = u32x4{0u, 0u, 0u, 0u};
                if (valid) {
                    const uint4 w = *reinterpret_cast<const uint4 *>(hist + b4);
                    v = u32x4{w.x, w.y, w.z, w.w};
                    __builtin_nontemporal_store(v, reinterpret_cast<u32x4 *>(out + h0 + b4));
                }
                if (a.sel_bits) select_words(h0 + base, valid, v);
            }
        }
    }
    if (!a.sel_bits) return;
    // the item's passing bins and members, summed over its slices
    sel_ms = wave_sum(sel_ms);
    if (lane == 0) {
        atomicAdd(sel_acc, sel_ne);
        atomicAdd(sel_acc + 1, sel_ms);
    }
    __syncthreads();
    if (tid == 0) {
        atomicAdd(reinterpret_cast<unsigned long long *>(a.sel_ne + j), (unsigned long long)sel_acc[0]);
        atomicAdd(reinterpret_cast<unsigned long long *>(a.sel_ms + j), (unsigned long long)sel_acc[1]);
    }
}

// ---------------------------------------------------------------- a3 - a5 fused
// Projection, histogram and enriched-bucket list without keys or counts in
// HBM.  Pass COUNT: the histogram of the (item, slice) in LDS, then its
// number of passing bins and their total size.  Pass EMIT (after a scan of
// those totals): the same histogram again; a block scan over the slice's bins
// gives every passing bin its bucket number and first member slot, the bucket
// records are written in key order, each passing bin's count is replaced in
// place by its first slot (non-passing bins by an all-ones sentinel), and a
// second sweep over the windows places every member with an LDS atomic add on
// its bin, whose returned value is the member's slot.  Members of a bucket are
// therefore complete but in no particular order.
struct HselArgs {
    HashArgs h;
    uint32_t s;
    int64_t *tot_b, *tot_m;          // [items * nslices]: passing bins and their members
    const int64_t *base_b, *base_m;  // [items * nslices]: their first bucket and member slot (EMIT)
    pm_bucket *buckets;
    uint32_t *members;
    int64_t cap_b, cap_m;
};

constexpr int kHselScanWords = 2 * kHashThreads;  // LDS words of the bin scan (per-thread totals)

template <bool U16>
__device__ __forceinline__ uint32_t hist_get(const uint32_t *hist, uint32_t bin)
{
    return U16 ? (hist[bin >> 1] >> ((bin & 1) << 4)) & 0xffffu : hist[bin];
}

template <bool U16>
__device__ __forceinline__ void hist_set(uint32_t *hist, uint32_t bin, uint32_t v)
{
    if (U16) {
        const uint32_t sh = (bin & 1) << 4;
        hist[bin >> 1] = (hist[bin >> 1] & ~(0xffffu << sh)) | ((v & 0xffffu) << sh);
    } else {
        hist[bin] = v;
    }
}

template <int A, int K, bool U16, bool EMIT>
__global__ void __launch_bounds__(kHashThreads) k_hsel(const HselArgs g)
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
    uint32_t *hist = smem;
    uint32_t *seq = smem + a.hist_words;
    int32_t *wst = reinterpret_cast<int32_t *>(seq + a.seq_cap);
    uint32_t *scan = reinterpret_cast<uint32_t *>(wst + a.off_cap);  // [kHselScanWords]
    const Staged st = stage_input<A>(a, j, seq, wst);
    for (int i = tid * 4; i < a.hist_words; i += kHashThreads * 4)
        *reinterpret_cast<uint4 *>(hist + i) = make_uint4(0, 0, 0, 0);
    __syncthreads();
    int pos[K];
    kept_positions<A, K>(mask, pos);
    const uint32_t slice_base = (uint32_t)slice * a.slice_bins;
    for_each_key<A, K>(a, st, pos, [&](int64_t, uint32_t key) {
        const uint32_t bin = key - slice_base;
        if (bin < a.slice_bins) hist_add<U16>(hist, bin);
    });
    __syncthreads();

    // the slice's valid bins, an even number per thread (whole u16 pairs)
    const uint64_t left = (uint64_t)a.nb - slice_base;
    const uint32_t nvalid = left < a.slice_bins ? (uint32_t)left : a.slice_bins;
    const uint32_t per = ((nvalid + kHashThreads - 1) / kHashThreads + 1) & ~1u;
    const uint32_t lo = min(tid * per, nvalid), hi = min(lo + per, nvalid);
    uint32_t nbk = 0, nmem = 0;
    for (uint32_t b = lo; b < hi; ++b) {
        const uint32_t c = hist_get<U16>(hist, b);
        if (c >= g.s && c > 0) {
            nbk += 1;
            nmem += c;
        }
    }
    if (!EMIT) {
        // totals of the (item, slice)
        const uint32_t tb = wave_sum(nbk), tm = wave_sum(nmem);
        if (lane_id() == 0) {
            scan[2 * (tid >> 6)] = tb;
            scan[2 * (tid >> 6) + 1] = tm;
        }
        __syncthreads();
        if (tid == 0) {
            int64_t sb = 0, sm = 0;
            for (int w = 0; w < kHashThreads / 64; ++w) {
                sb += scan[2 * w];
                sm += scan[2 * w + 1];
            }
            g.tot_b[e] = sb;
            g.tot_m[e] = sm;
        }
        return;
    }
    // exclusive scan of the per-thread (buckets, members) over the workgroup
    scan[tid] = nbk;
    scan[kHashThreads + tid] = nmem;
    __syncthreads();
    for (int o = 1; o < kHashThreads; o <<= 1) {
        const uint32_t ub = tid >= o ? scan[tid - o] : 0u, um = tid >= o ? scan[kHashThreads + tid - o] : 0u;
        __syncthreads();
        scan[tid] += ub;
        scan[kHashThreads + tid] += um;
        __syncthreads();
    }
    uint32_t bi = scan[tid] - nbk, mi = scan[kHashThreads + tid] - nmem;
    const int64_t bb = g.base_b[e], mb = g.base_m[e];
    constexpr uint32_t kNone = U16 ? 0xffffu : 0xffffffffu;
    for (uint32_t b = lo; b < hi; ++b) {
        const uint32_t c = hist_get<U16>(hist, b);
        if (c >= g.s && c > 0) {
            const int64_t idx = bb + bi;
            if (idx < g.cap_b)
                g.buckets[idx] = pm_bucket{(uint32_t)j, slice_base + b, c, (uint32_t)(mb + mi)};
            hist_set<U16>(hist, b, mi);
            bi += 1;
            mi += c;
        } else {
            hist_set<U16>(hist, b, kNone);
        }
    }
    __syncthreads();
    // members: each window of a passing bin takes the bin's next slot
    for_each_key<A, K>(a, st, pos, [&](int64_t w, uint32_t key) {
        const uint32_t bin = key - slice_base;
        if (bin < a.slice_bins && hist_get<U16>(hist, bin) != kNone) {
            uint32_t slot;
            if (U16) slot = (atomicAdd(hist + (bin >> 1), 1u << ((bin & 1) << 4)) >> ((bin & 1) << 4)) & 0xffffu;
            else slot = atomicAdd(hist + bin, 1u);
            const int64_t ms = mb + slot;
            if (ms < g.cap_m) g.members[ms] = (uint32_t)w;
        }
    });
}

template <int A, int K, int HIST>
static int launch_hash(const HashArgs &a, size_t lds, int blocks, hipStream_t st)
{
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)k_hash<A, K, HIST>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, device_lds_bytes());
        (void)hipGetLastError();  // an unsupported attribute must not poison the launch check
        attr_set = true;
    }
    hipLaunchKernelGGL((k_hash<A, K, HIST>), dim3(blocks), dim3(kHashThreads), lds, st, a);
    PM_LAUNCHED();
    return PM_OK;
}

template <int A, int K, bool U16, bool EMIT>
static int launch_hsel(const HselArgs &g, size_t lds, int blocks, hipStream_t st)
{
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)k_hsel<A, K, U16, EMIT>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, device_lds_bytes());
        (void)hipGetLastError();
        attr_set = true;
    }
    hipLaunchKernelGGL((k_hsel<A, K, U16, EMIT>), dim3(blocks), dim3(kHashThreads), lds, st, g);
    PM_LAUNCHED();
    return PM_OK;
}

template <int K>
static int dispatch_hsel(int alphabet, int k, bool u16, bool emit, const HselArgs &g, size_t lds, int blocks,
                         hipStream_t st)
{
    constexpr int KMAX = 12;  // |Sigma|^k within the LDS histogram's slices
    if constexpr (K > KMAX) {
        return fail(PM_ERANGE, "k=%d not supported by the fused selection", k);
    } else {
        if (k != K) return dispatch_hsel<K + 1>(alphabet, k, u16, emit, g, lds, blocks, st);
        if (alphabet == 4) {
            if (u16) return emit ? launch_hsel<4, K, true, true>(g, lds, blocks, st)
                                 : launch_hsel<4, K, true, false>(g, lds, blocks, st);
            return emit ? launch_hsel<4, K, false, true>(g, lds, blocks, st)
                        : launch_hsel<4, K, false, false>(g, lds, blocks, st);
        }
        if constexpr (K <= 5) {
            if (u16) return emit ? launch_hsel<20, K, true, true>(g, lds, blocks, st)
                                 : launch_hsel<20, K, true, false>(g, lds, blocks, st);
            return emit ? launch_hsel<20, K, false, true>(g, lds, blocks, st)
                        : launch_hsel<20, K, false, false>(g, lds, blocks, st);
        }
        return fail(PM_ERANGE, "k=%d not supported by the fused selection for protein", k);
    }
}

// run-time (alphabet, k, count-table width) -> compile-time kernel
template <int H, int A, int K>
static int launch_hist(int hist, const HashArgs &a, size_t lds, int blocks, hipStream_t st)
{
    if constexpr (H >= kHistModes) {
        return fail(PM_EINVAL, "unknown count-table width %d", hist);
    } else {
        if (hist != H) return launch_hist<H + 1, A, K>(hist, a, lds, blocks, st);
        return launch_hash<A, K, H>(a, lds, blocks, st);
    }
}

template <int K>
static int dispatch_hash(int alphabet, int k, int hist, const HashArgs &a, size_t lds, int blocks, hipStream_t st)
{
    constexpr int KMAX = 16;
    if constexpr (K > KMAX) {
        return fail(PM_ERANGE, "k=%d not supported", k);
    } else {
        if (k != K) return dispatch_hash<K + 1>(alphabet, k, hist, a, lds, blocks, st);
        if (alphabet == 4) return launch_hist<kHist16, 4, K>(hist, a, lds, blocks, st);
        if constexpr (K <= 7) return launch_hist<kHist16, 20, K>(hist, a, lds, blocks, st);
        return fail(PM_ERANGE, "k=%d not supported for protein", k);
    }
}

}  // namespace pm

using namespace pm;

extern "C" int64_t pm_packed_words(int32_t alphabet, int64_t n_total)
{
    if (alphabet != 4 && alphabet != 20) return -1;
    const int per = alphabet == 4 ? 16 : 6;
    return (n_total + per - 1) / per + 4;
}

extern "C" int pm_pack(int32_t alphabet, const uint8_t *ascii, int64_t n_total, uint32_t *packed,
                       uint32_t *status, void *stream)
{
    clear_error();
    if (alphabet != 4 && alphabet != 20) return fail(PM_EINVAL, "alphabet must be 4 or 20");
    if (n_total < 0 || (n_total > 0 && !ascii) || !packed) return fail(PM_EINVAL, "bad buffers");
    const int64_t nw = pm_packed_words(alphabet, n_total);
    const int threads = 256;
    const int64_t blocks = (nw + threads - 1) / threads;
    hipLaunchKernelGGL(k_pack, dim3((unsigned)blocks), dim3(threads), 0, as_stream(stream), alphabet,
                       ascii, n_total, packed, nw, status);
    PM_LAUNCHED();
    return PM_OK;
}

// LDS layout for the largest instance (staged input, histogram slices):
// returns the dynamic LDS bytes, or 0 after fail().  per_word: counts per
// 32-bit LDS word (1, 2 or 4); extra: further fixed LDS words; balance: split
// a whole-trial histogram that would leave its workgroup alone on a CU into
// two slices.
static size_t hash_layout(HashArgs &a, bool hist, int per_word, int64_t nw_max, int t_max, int extra, bool balance)
{
    const int lds_max = device_lds_bytes();
    const int64_t sw = staged_words(a.A, nw_max);
    a.off_cap = (t_max + 1) * 4 <= 8 * 1024 ? t_max + 1 : 0;
    // protein bytes are read only by the staged path, which needs the
    // window starts staged too
    a.seq_cap = sw * 4 <= 48 * 1024 && (a.A == 4 || a.off_cap) ? (int)sw : 0;
    const int fixed = (a.seq_cap + a.off_cap + extra) * 4;
    if (hist) {
        const int64_t need_words = (a.nb + per_word - 1) / per_word;
        int64_t budget = (lds_max - fixed) / 4;
        budget &= ~int64_t(3);
        if (budget < 1024) {
            fail(PM_ERANGE, "input too large for the LDS budget");
            return 0;
        }
        int64_t hw = std::min<int64_t>(need_words, budget);
        // a whole-trial histogram that fits one workgroup but leaves it alone on
        // its CU goes into two balanced slices instead, so that two workgroups
        // share a CU and one's key pass overlaps the other's count write-out
        // (each slice recomputes the trial's keys; measured 11% faster on the
        // (18,6) workload's 128 KB histograms)
        const int64_t half = ((int64_t)lds_max / 2 - fixed) / 4;
        int64_t cap = budget;
        if (balance && need_words <= budget && need_words > half && (need_words + 1) / 2 <= half && half >= 1024) {
            hw = (need_words + 1) / 2;
            cap = half;
        }
        hw = (hw + 3) & ~int64_t(3);
        if (hw > budget) hw = budget;
        if (a.sel_bits) {
            // the selection's bitmap: every slice and every u32 recount pass
            // a whole number of 256-bin groups (budget >= 1024 words)
            const int64_t up = (hw + 255) & ~int64_t(255);
            hw = up <= cap ? up : hw & ~int64_t(255);
        }
        a.hist_words = (int)hw;
        a.slice_bins = (uint32_t)(per_word * hw);
        a.nslices = (int)((a.nb + a.slice_bins - 1) / a.slice_bins);
    } else {
        a.hist_words = 0;
        a.slice_bins = 0;
        a.nslices = 1;
    }
    return (size_t)a.hist_words * 4 + fixed;
}

// sizes the LDS for the largest instance and launches one workgroup per
// (item, slice)
static int hash_launch(HashArgs &a, int A, int32_t items, int64_t x_max, int64_t nw_max, int t_max,
                       hipStream_t st)
{
    // the count width giving the fewest slices (each slice recomputes its
    // trial's keys), then the most workgroups per CU (one's key pass overlaps
    // another's count write-out), then the widest: no check for u32, nor for
    // u16 below 65 536 windows
    int hist = kHist16, per_word = 2;
    if (a.counts) {
        int best_slices = 0x7fffffff, best_wgs = 0;
        for (const int pw : {1, 2, 4, 8}) {
            HashArgs probe = a;
            const size_t bytes = hash_layout(probe, true, pw, nw_max, t_max, kHashFlagWords, true);
            if (!bytes) continue;
            const int wgs = std::min((int)(device_lds_bytes() / bytes), 2048 / kHashThreads);
            if (probe.nslices < best_slices || (probe.nslices == best_slices && wgs > best_wgs)) {
                best_slices = probe.nslices;
                best_wgs = wgs;
                per_word = pw;
            }
        }
        hist = per_word == 1   ? kHist32
               : per_word == 8 ? kHist4
               : per_word == 4 ? kHist8
               : x_max < 65536 ? kHist16
                               : kHist16Check;
    }
    const size_t lds = hash_layout(a, a.counts != nullptr, per_word, nw_max, t_max, kHashFlagWords, true);
    if (!lds) return PM_ERANGE;
    const int64_t blocks = (int64_t)items * a.nslices;
    if (blocks > 0x7fffffff) return fail(PM_ERANGE, "too many trials x slices");
    return dispatch_hash<1>(A, a.k, hist, a, lds, (int)blocks, st);
}

// ---- fused selection: workspace of per-(item, slice) totals and bases
static int64_t hsel_entries(HashArgs a, int32_t items, int64_t x_max, int64_t nw_max, int t_max)
{
    if (!hash_layout(a, true, x_max < 65536 ? 2 : 1, nw_max, t_max, kHselScanWords, false)) return -1;
    return (int64_t)items * a.nslices;
}

static size_t hsel_ws_bytes(int64_t entries) { return entries < 0 ? 0 : (size_t)entries * 4 * sizeof(int64_t) + 256; }

static int check_hsel_args(int A, int l, int k, const uint32_t *masks, int64_t items, const int64_t *n_out,
                           pm_bucket *buckets, int64_t cap_b, uint32_t *members, int64_t cap_m, void *ws)
{
    if (k < 1 || k > l) return fail(PM_EINVAL, "need 1 <= k <= l (k=%d, l=%d)", k, l);
    if (items < 1) return fail(PM_EINVAL, "need at least one trial");
    if (!masks || !n_out || !ws) return fail(PM_EINVAL, "masks, n_out and ws are required");
    if (cap_b < 0 || cap_m < 0) return fail(PM_EINVAL, "negative capacity");
    if ((cap_b > 0 && !buckets) || (cap_m > 0 && !members)) return fail(PM_EINVAL, "NULL output with a non-zero capacity");
    if (cap_m > 0xffffffffll) return fail(PM_ERANGE, "cap_members must be below 2^32");
    return PM_OK;
}

// count-table (LDS histogram) selection for DNA k <= 12 and protein k <= 5;
// larger key spaces go to the sorted selection
static bool dense_sel(int A, int k) { return (A == 4 && k <= 12) || (A == 20 && k <= 5); }

static int hsel_run(HashArgs &a, int A, int32_t items, int64_t x_max, int64_t nw_max, int t_max, uint32_t s,
                    pm_bucket *buckets, int64_t cap_b, uint32_t *members, int64_t cap_m, int64_t *n_out, void *ws,
                    size_t ws_bytes, hipStream_t st)
{
    const size_t lds = hash_layout(a, true, x_max < 65536 ? 2 : 1, nw_max, t_max, kHselScanWords, false);
    if (!lds) return PM_ERANGE;
    const int64_t entries = (int64_t)items * a.nslices;
    if (entries > 0x7fffffff) return fail(PM_ERANGE, "too many trials x slices");
    if (ws_bytes < hsel_ws_bytes(entries)) return fail(PM_EINVAL, "workspace of %zu bytes, need %zu", ws_bytes,
                                                      hsel_ws_bytes(entries));
    int64_t *w = static_cast<int64_t *>(ws);
    HselArgs g{};
    g.h = a;
    g.s = s;
    g.tot_b = w;
    g.tot_m = w + entries;
    g.base_b = w + 2 * entries;
    g.base_m = w + 3 * entries;
    g.buckets = buckets;
    g.members = members;
    g.cap_b = cap_b;
    g.cap_m = cap_m;
    const bool u16 = x_max < 65536;
    if (int rc = dispatch_hsel<1>(A, a.k, u16, false, g, lds, (int)entries, st)) return rc;
    const TotScan ts{g.tot_b, g.tot_m, w + 2 * entries, w + 3 * entries, entries, cap_b, cap_m, n_out, a.status};
    if (int rc = launch_tot_scan(ts, st)) return rc;
    if (cap_b == 0 && cap_m == 0) return PM_OK;  // sizing only
    return dispatch_hsel<1>(A, a.k, u16, true, g, lds, (int)entries, st);
}

static int check_hash_args(int A, int l, int k, const uint32_t *masks, int64_t items, const uint32_t *keys,
                           const uint32_t *counts)
{
    if (k < 1 || k > l) return fail(PM_EINVAL, "need 1 <= k <= l (k=%d, l=%d)", k, l);
    if (items < 0) return fail(PM_EINVAL, "m must be >= 0");
    if (!masks && items > 0) return fail(PM_EINVAL, "masks is NULL");
    if (!keys && !counts) return fail(PM_EINVAL, "keys and counts are both NULL");
    if ((A == 4 && k > 16) || (A == 20 && k > 7))
        return fail(PM_ERANGE, "|Sigma|^k must stay below 2^32 (k=%d)", k);
    if (counts && ipow(A, k) > (1ll << 24))
        return fail(PM_ERANGE, "|Sigma|^k = %lld bins is above 2^24", (long long)ipow(A, k));
    return PM_OK;
}

extern "C" int projection_hash(const pm_seqs *S, int32_t l, int32_t k, const uint32_t *masks,
                               int32_t m, uint32_t *keys, uint32_t *counts, uint32_t *status,
                               void *stream)
{
    clear_error();
    int rc = check_seqs(S, l);
    if (rc) return rc;
    const int A = S->alphabet;
    if ((rc = check_hash_args(A, l, k, masks, m, keys, counts))) return rc;
    if (m == 0) return PM_OK;
    HashArgs a{};
    a.A = A;
    a.one = inst_of(S, l);
    a.masks = masks;
    a.keys = keys;
    a.counts = counts;
    a.status = status;
    a.nb = ipow(A, k);
    a.l = l;
    a.k = k;
    return hash_launch(a, A, m, a.one.x, pm_packed_words(A, S->n_total), S->t, as_stream(stream));
}

extern "C" int projection_hash_batch(const pm_batch *B, const uint32_t *masks, uint32_t *keys,
                                     uint32_t *counts, uint32_t *status, void *stream)
{
    clear_error();
    BatchInfo info;
    int rc = check_batch(B, &info);
    if (rc) return rc;
    const int A = B->alphabet;
    if ((rc = check_hash_args(A, B->l, B->k, masks, B->items, keys, counts))) return rc;
    HashArgs a{};
    a.A = A;
    a.inst = B->inst;
    a.item_inst = B->item_inst;
    a.masks = masks;
    a.keys = keys;
    a.counts = counts;
    a.status = status;
    a.nb = ipow(A, B->k);
    a.l = B->l;
    a.k = B->k;
    return hash_launch(a, A, B->items, info.x_max, info.nw_max, info.t_max, as_stream(stream));
}

// the hash launch of projection_hash_select: keys and counts as
// projection_hash writes them, and the selection's bitmap and totals
static int hash_counted(HashArgs &a, int A, int32_t items, int64_t x_max, int64_t nw_max, int t_max, uint32_t s,
                        void *ws, hipStream_t st)
{
    SelCounted c;
    if (int rc = select_counted_prepare(ws, items, A, a.k, &c, st)) return rc;
    a.sel_bits = c.bits;
    a.sel_ne = c.ne;
    a.sel_ms = c.ms;
    a.sel_nwb = c.nwb;
    a.sel_smin = s > 1u ? s : 1u;  // s = 0 selects like s = 1
    return hash_launch(a, A, items, x_max, nw_max, t_max, st);
}

extern "C" int projection_hash_select(const pm_seqs *S, int32_t l, int32_t k, const uint32_t *masks, int32_t m,
                                      uint32_t *keys, uint32_t *counts, uint32_t s, pm_bucket *buckets,
                                      int64_t cap_buckets, uint32_t *members, int64_t cap_members, int64_t *n_out,
                                      void *ws, size_t ws_bytes, uint32_t *status, void *stream)
{
    clear_error();
    int rc = check_seqs(S, l);
    if (rc) return rc;
    const int A = S->alphabet;
    if ((rc = check_hash_args(A, l, k, masks, m, keys, counts))) return rc;
    if ((rc = check_select_ws(A, k, m, keys, counts, n_out, ws, ws_bytes, buckets, cap_buckets, members,
                              cap_members)))
        return rc;
    HashArgs a{};
    a.A = A;
    a.one = inst_of(S, l);
    a.masks = masks;
    a.keys = keys;
    a.counts = counts;
    a.status = status;
    a.nb = ipow(A, k);
    a.l = l;
    a.k = k;
    const hipStream_t st = as_stream(stream);
    if ((rc = hash_counted(a, A, m, a.one.x, pm_packed_words(A, S->n_total), S->t, s, ws, st))) return rc;
    return select_counted(a.one, nullptr, nullptr, A, k, keys, counts, m, s, buckets, cap_buckets, members,
                          cap_members, n_out, ws, status, a.one.x, st);
}

extern "C" int projection_hash_select_batch(const pm_batch *B, const uint32_t *masks, uint32_t *keys,
                                            uint32_t *counts, uint32_t s, pm_bucket *buckets, int64_t cap_buckets,
                                            uint32_t *members, int64_t cap_members, int64_t *n_out, void *ws,
                                            size_t ws_bytes, uint32_t *status, void *stream)
{
    clear_error();
    BatchInfo info;
    int rc = check_batch(B, &info);
    if (rc) return rc;
    const int A = B->alphabet;
    if ((rc = check_hash_args(A, B->l, B->k, masks, B->items, keys, counts))) return rc;
    if ((rc = check_select_ws(A, B->k, B->items, keys, counts, n_out, ws, ws_bytes, buckets, cap_buckets, members,
                              cap_members)))
        return rc;
    HashArgs a{};
    a.A = A;
    a.inst = B->inst;
    a.item_inst = B->item_inst;
    a.masks = masks;
    a.keys = keys;
    a.counts = counts;
    a.status = status;
    a.nb = ipow(A, B->k);
    a.l = B->l;
    a.k = B->k;
    const hipStream_t st = as_stream(stream);
    if ((rc = hash_counted(a, A, B->items, info.x_max, info.nw_max, info.t_max, s, ws, st))) return rc;
    return select_counted(a.one, B->inst, B->item_inst, A, B->k, keys, counts, B->items, s, buckets, cap_buckets,
                          members, cap_members, n_out, ws, status, info.x_max, st);
}

extern "C" size_t pm_hash_select_workspace(const pm_seqs *S, int32_t l, int32_t k, int32_t m)
{
    clear_error();
    if (check_seqs(S, l) != PM_OK || k < 1 || k > l || m < 1) return 0;
    const int A = S->alphabet;
    const int64_t x = num_windows(S, l), nw = pm_packed_words(A, S->n_total);
    if (!dense_sel(A, k)) return hsort_check_k(A, k) ? 0 : hsort_workspace(A, l, k, m, x, nw, S->t);
    HashArgs a{};
    a.A = A;
    a.nb = ipow(A, k);
    return hsel_ws_bytes(hsel_entries(a, m, x, nw, S->t));
}

extern "C" size_t pm_sort_select_workspace(const pm_seqs *S, int32_t l, int32_t k, int32_t m)
{
    clear_error();
    if (check_seqs(S, l) != PM_OK || k < 1 || k > l || m < 1 || hsort_check_k(S->alphabet, k)) return 0;
    return hsort_workspace(S->alphabet, l, k, m, num_windows(S, l), pm_packed_words(S->alphabet, S->n_total), S->t);
}

extern "C" size_t pm_hash_select_batch_workspace(const pm_batch *B)
{
    clear_error();
    BatchInfo info;
    if (check_batch(B, &info) != PM_OK) return 0;
    const int A = B->alphabet;
    if (!dense_sel(A, B->k))
        return hsort_check_k(A, B->k) ? 0 : hsort_workspace(A, B->l, B->k, B->items, info.x_max, info.nw_max, info.t_max);
    HashArgs a{};
    a.A = A;
    a.nb = ipow(A, B->k);
    return hsel_ws_bytes(hsel_entries(a, B->items, info.x_max, info.nw_max, info.t_max));
}

extern "C" size_t pm_sort_select_batch_workspace(const pm_batch *B)
{
    clear_error();
    BatchInfo info;
    if (check_batch(B, &info) != PM_OK || hsort_check_k(B->alphabet, B->k)) return 0;
    return hsort_workspace(B->alphabet, B->l, B->k, B->items, info.x_max, info.nw_max, info.t_max);
}

static int hash_select_one(const pm_seqs *S, int32_t l, int32_t k, const uint32_t *masks, int32_t m, uint32_t s,
                           pm_bucket *buckets, int64_t cap_buckets, uint32_t *members, int64_t cap_members,
                           int64_t *n_out, void *ws, size_t ws_bytes, uint32_t *status, void *stream, bool sorted)
{
    clear_error();
    int rc = check_seqs(S, l);
    if (rc) return rc;
    const int A = S->alphabet;
    if ((rc = check_hsel_args(A, l, k, masks, m, n_out, buckets, cap_buckets, members, cap_members, ws))) return rc;
    HashArgs a{};
    a.A = A;
    a.one = inst_of(S, l);
    a.masks = masks;
    a.status = status;
    a.nb = ipow(A, k);
    a.l = l;
    a.k = k;
    const int64_t nw = pm_packed_words(A, S->n_total);
    if (!sorted && dense_sel(A, k))
        return hsel_run(a, A, m, a.one.x, nw, S->t, s, buckets, cap_buckets, members, cap_members, n_out, ws,
                        ws_bytes, as_stream(stream));
    return hsort_run(a, A, m, a.one.x, nw, S->t, s, buckets, cap_buckets, members, cap_members, n_out, ws, ws_bytes,
                     as_stream(stream));
}

static int hash_select_batch(const pm_batch *B, const uint32_t *masks, uint32_t s, pm_bucket *buckets,
                             int64_t cap_buckets, uint32_t *members, int64_t cap_members, int64_t *n_out, void *ws,
                             size_t ws_bytes, uint32_t *status, void *stream, bool sorted)
{
    clear_error();
    BatchInfo info;
    int rc = check_batch(B, &info);
    if (rc) return rc;
    const int A = B->alphabet;
    if ((rc = check_hsel_args(A, B->l, B->k, masks, B->items, n_out, buckets, cap_buckets, members, cap_members, ws)))
        return rc;
    HashArgs a{};
    a.A = A;
    a.inst = B->inst;
    a.item_inst = B->item_inst;
    a.masks = masks;
    a.status = status;
    a.nb = ipow(A, B->k);
    a.l = B->l;
    a.k = B->k;
    if (!sorted && dense_sel(A, B->k))
        return hsel_run(a, A, B->items, info.x_max, info.nw_max, info.t_max, s, buckets, cap_buckets, members,
                        cap_members, n_out, ws, ws_bytes, as_stream(stream));
    return hsort_run(a, A, B->items, info.x_max, info.nw_max, info.t_max, s, buckets, cap_buckets, members,
                     cap_members, n_out, ws, ws_bytes, as_stream(stream));
}

extern "C" int bucket_hash_select(const pm_seqs *S, int32_t l, int32_t k, const uint32_t *masks, int32_t m,
                                  uint32_t s, pm_bucket *buckets, int64_t cap_buckets, uint32_t *members,
                                  int64_t cap_members, int64_t *n_out, void *ws, size_t ws_bytes, uint32_t *status,
                                  void *stream)
{
    return hash_select_one(S, l, k, masks, m, s, buckets, cap_buckets, members, cap_members, n_out, ws, ws_bytes,
                           status, stream, false);
}

extern "C" int bucket_sort_select(const pm_seqs *S, int32_t l, int32_t k, const uint32_t *masks, int32_t m,
                                  uint32_t s, pm_bucket *buckets, int64_t cap_buckets, uint32_t *members,
                                  int64_t cap_members, int64_t *n_out, void *ws, size_t ws_bytes, uint32_t *status,
                                  void *stream)
{
    return hash_select_one(S, l, k, masks, m, s, buckets, cap_buckets, members, cap_members, n_out, ws, ws_bytes,
                           status, stream, true);
}

extern "C" int bucket_hash_select_batch(const pm_batch *B, const uint32_t *masks, uint32_t s, pm_bucket *buckets,
                                        int64_t cap_buckets, uint32_t *members, int64_t cap_members, int64_t *n_out,
                                        void *ws, size_t ws_bytes, uint32_t *status, void *stream)
{
    return hash_select_batch(B, masks, s, buckets, cap_buckets, members, cap_members, n_out, ws, ws_bytes, status,
                             stream, false);
}

extern "C" int bucket_sort_select_batch(const pm_batch *B, const uint32_t *masks, uint32_t s, pm_bucket *buckets,
                                        int64_t cap_buckets, uint32_t *members, int64_t cap_members, int64_t *n_out,
                                        void *ws, size_t ws_bytes, uint32_t *status, void *stream)
{
    return hash_select_batch(B, masks, s, buckets, cap_buckets, members, cap_members, n_out, ws, ws_bytes, status,
                             stream, true);
}

// ---- allocation-free form of the fused selection
// The per-(trial, slice) totals and bases live in a fixed device array instead
// of a caller workspace.  Its host-side name is not a device address: every
// use goes through the address hipGetSymbolAddress returns on each device.
constexpr size_t kHselScratchBytes = size_t(8) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kHselScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

static int scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(PM_EDEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(PM_EDEVICE, "device %d beyond the %d this library tracks", dev,
                                                  kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PM_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PM_OK;
}

extern "C" size_t pm_hash_select_scratch_bytes(void) { return kHselScratchBytes; }

extern "C" int bucket_hash_select_noalloc(const pm_seqs *S, int32_t l, int32_t k, const uint32_t *masks, int32_t m,
                                          uint32_t s, pm_bucket *buckets, int64_t cap_buckets, uint32_t *members,
                                          int64_t cap_members, int64_t *n_out, uint32_t *status, void *stream)
{
    clear_error();
    int rc = check_seqs(S, l);
    if (rc) return rc;
    const int A = S->alphabet;
    // the scratch stands in for the workspace: pass its address as non-NULL
    // only after the size check below, so the argument check sees a workspace
    if ((rc = check_hsel_args(A, l, k, masks, m, n_out, buckets, cap_buckets, members, cap_members,
                              reinterpret_cast<void *>(uintptr_t(1)))))
        return rc;
    HashArgs a{};
    a.A = A;
    a.one = inst_of(S, l);
    a.masks = masks;
    a.status = status;
    a.nb = ipow(A, k);
    a.l = l;
    a.k = k;
    const int64_t nw = pm_packed_words(A, S->n_total);
    const bool dense = dense_sel(A, k);
    if (!dense && (rc = hsort_check_k(A, k))) return rc;
    const size_t need = dense ? hsel_ws_bytes(hsel_entries(a, m, a.one.x, nw, S->t))
                              : hsort_workspace(A, l, k, m, a.one.x, nw, S->t);
    if (need == 0) return fail(PM_ERANGE, "this instance does not fit the fused selection's LDS layout");
    if (need > kHselScratchBytes)
        return fail(PM_ERANGE, "%d trials need %zu bytes of scratch; the fixed scratch holds %zu (at most %zu "
                               "trial-slices)",
                    m, need, kHselScratchBytes, (kHselScratchBytes - 256) / (4 * sizeof(int64_t)));
    void *ws = nullptr;
    if ((rc = scratch_address(&ws))) return rc;
    if (dense)
        return hsel_run(a, A, m, a.one.x, nw, S->t, s, buckets, cap_buckets, members, cap_members, n_out, ws,
                        kHselScratchBytes, as_stream(stream));
    return hsort_run(a, A, m, a.one.x, nw, S->t, s, buckets, cap_buckets, members, cap_members, n_out, ws,
                     kHselScratchBytes, as_stream(stream));
}
