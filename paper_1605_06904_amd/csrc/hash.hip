// a1 (encode + pack) and a3/a4 (projection, keys, bucket histogram) on gfx950.
//
// Sec. 6 of the paper maps letters to integers and projects/hashes one l-mer
// per GPU thread.  Here one workgroup owns one trial (and one slice of the
// key range when the |Sigma|^k histogram does not fit in LDS): it stages the
// packed input (a few KB) in LDS, builds keys from LDS windows, writes them
// with coalesced stores and counts them in an LDS histogram with
// wave-aggregated atomics, then streams the histogram out as dense u32 counts.
#include <algorithm>

#include "pm_common.h"

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
struct HashArgs {
    pm_inst one;               // the instance, when inst is NULL
    const pm_inst *inst;       // batch: instance table, or NULL
    const int32_t *item_inst;  // batch: instance of every trial item
    const uint32_t *masks;
    uint32_t *keys;
    uint32_t *counts;
    uint32_t *status;
    int64_t nb;          // |Sigma|^k
    int l, k;
    int nslices;         // key-range slices per trial
    uint32_t slice_bins; // bins per slice (multiple of 4)
    int hist_words;      // LDS words of histogram
    int seq_cap;         // LDS words reserved for the packed input (0: read from global)
    int off_cap;         // LDS window starts reserved, t + 1 (0: read offsets from global)
};

constexpr int kHashThreads = 1024;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int A, int K, bool U16>
__global__ void __launch_bounds__(kHashThreads) k_hash(const HashArgs a)
{
    extern __shared__ __align__(16) uint32_t smem[];
    const int slice = blockIdx.x % a.nslices;
    const int j = blockIdx.x / a.nslices;
    const int tid = threadIdx.x;
    const pm_inst I = a.inst ? a.inst[a.item_inst[j]] : a.one;
    const int64_t x = I.x;
    const int seq_words = a.seq_cap ? (int)(A == 4 ? (I.n_total + 15) / 16 + 4 : (I.n_total + 5) / 6 + 4) : 0;

    const uint32_t mask = a.masks[j];
    const uint32_t lmask = a.l == 32 ? 0xffffffffu : ((1u << a.l) - 1u);
    if (__popc(mask) != a.k || (mask & ~lmask)) {
        if (tid == 0 && slice == 0 && a.status) atomicOr(a.status, PM_STATUS_BAD_MASK);
        return;
    }

    uint32_t *hist = smem;
    uint32_t *seq = smem + a.hist_words;
    int32_t *wst = reinterpret_cast<int32_t *>(seq + a.seq_cap);  // window number of each sequence start

    for (int i = tid; i < seq_words; i += kHashThreads) seq[i] = I.packed[i];
    if (a.off_cap)
        for (int i = tid; i <= I.t; i += kHashThreads) wst[i] = (int32_t)(I.offsets[i] - (int64_t)i * (a.l - 1));
    if (a.counts)
        for (int i = tid * 4; i < a.hist_words; i += kHashThreads * 4)
            *reinterpret_cast<uint4 *>(hist + i) = make_uint4(0, 0, 0, 0);
    __syncthreads();

    // kept positions, ascending (uniform across the workgroup): the shift of
    // each kept position's 2-bit field in the 64-bit window (DNA), or the
    // position itself (protein)
    int pos[K];
    {
        uint32_t mm = mask;
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const int p = __builtin_ctz(mm);
            pos[q] = A == 4 ? 62 - 2 * p : p;
            mm &= mm - 1;
        }
    }

    const uint32_t slice_base = (uint32_t)slice * a.slice_bins;  // |Sigma|^k <= 2^24
    const int64_t kw0 = x * slice / a.nslices, kw1 = x * (slice + 1) / a.nslices;
    uint32_t *keys_j = a.keys ? a.keys + I.key_base + (int64_t)(j - I.first_item) * x : nullptr;
    auto count = [&](uint32_t key) {
        const uint32_t bin = key - slice_base;
        if (bin < a.slice_bins) {
            if (U16) atomicAdd(hist + (bin >> 1), 1u << ((bin & 1) << 4));
            else atomicAdd(hist + bin, 1u);
        }
    };

    if (a.seq_cap && a.off_cap) {
        // staged input: every read below is an LDS read, all indices 32-bit
        // (n_total < 2^31)
        const uint32_t x32 = (uint32_t)x, lm1 = (uint32_t)(a.l - 1);
        const uint32_t k0 = (uint32_t)kw0, k1 = (uint32_t)kw1;
        int i = 0;
        for (uint32_t w = tid; w < x32; w += kHashThreads) {
            while ((int32_t)w >= wst[i + 1]) ++i;
            const uint32_t P = w + (uint32_t)i * lm1;
            uint32_t key = 0;
            if (A == 4) {
                const uint32_t wi = P >> 4, r = (P & 15u) << 1;
                const uint32_t w0 = seq[wi], w1 = seq[wi + 1], w2 = seq[wi + 2];
                const uint32_t hi = (uint32_t)((((uint64_t)w0 << 32) | w1) >> (32 - r));
                const uint32_t lo = (uint32_t)((((uint64_t)w1 << 32) | w2) >> (32 - r));
                const uint64_t win = ((uint64_t)hi << 32) | lo;
#pragma unroll
                for (int q = 0; q < K; ++q) key = (key << 2) | ((uint32_t)(win >> pos[q]) & 3u);
            } else {
#pragma unroll
                for (int q = 0; q < K; ++q) {
                    const uint32_t g = P + (uint32_t)pos[q];
                    const uint32_t qq = div6(g);
                    key = key * 20u + ((seq[qq] >> (27 - 5 * (g - 6u * qq))) & 31u);
                }
            }
            if (keys_j && w >= k0 && w < k1) __builtin_nontemporal_store(key, keys_j + w);
            if (a.counts) count(key);
        }
    } else {
        // large instances: packed input and offsets read from global memory
        const uint32_t *W = a.seq_cap ? seq : I.packed;
        const int64_t *O = I.offsets;
        const int64_t lm1 = a.l - 1;
        int i = 0;
        for (int64_t w = tid; w < x; w += kHashThreads) {
            while (w >= O[i + 1] - (int64_t)(i + 1) * lm1) ++i;
            const int64_t P = w + (int64_t)i * lm1;
            uint32_t key = 0;
            if (A == 4) {
                uint32_t hi, lo;
                dna_window(W, P, hi, lo);
                const uint64_t win = ((uint64_t)hi << 32) | lo;
#pragma unroll
                for (int q = 0; q < K; ++q) key = (key << 2) | ((uint32_t)(win >> pos[q]) & 3u);
            } else {
#pragma unroll
                for (int q = 0; q < K; ++q) key = key * 20u + prot_sym(W, P + pos[q]);
            }
            if (keys_j && w >= kw0 && w < kw1) __builtin_nontemporal_store(key, keys_j + w);
            if (a.counts) count(key);
        }
    }
    if (!a.counts) return;
    __syncthreads();

    const uint64_t left = (uint64_t)a.nb - slice_base;
    const uint32_t nvalid = left < a.slice_bins ? (uint32_t)left : a.slice_bins;  // multiple of 4
    uint32_t *out = a.counts + (int64_t)j * a.nb + slice_base;
    for (uint32_t b4 = tid * 4; b4 < nvalid; b4 += kHashThreads * 4) {
        uint4 v;
        if (U16) {
            const uint32_t w0 = hist[b4 >> 1], w1 = hist[(b4 >> 1) + 1];
            v = make_uint4(w0 & 0xffffu, w0 >> 16, w1 & 0xffffu, w1 >> 16);
        } else {
            v = *reinterpret_cast<const uint4 *>(hist + b4);
        }
        __builtin_nontemporal_store(u32x4{v.x, v.y, v.z, v.w}, reinterpret_cast<u32x4 *>(out + b4));
    }
}

template <int A, int K, bool U16>
static int launch_hash(const HashArgs &a, size_t lds, int blocks, hipStream_t st)
{
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)k_hash<A, K, U16>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, device_lds_bytes());
        (void)hipGetLastError();  // an unsupported attribute must not poison the launch check
        attr_set = true;
    }
    hipLaunchKernelGGL((k_hash<A, K, U16>), dim3(blocks), dim3(kHashThreads), lds, st, a);
    PM_LAUNCHED();
    return PM_OK;
}

// run-time (alphabet, k, histogram width) -> compile-time kernel
template <int K>
static int dispatch_hash(int alphabet, int k, bool u16, const HashArgs &a, size_t lds, int blocks, hipStream_t st)
{
    constexpr int KMAX = 16;
    if constexpr (K > KMAX) {
        return fail(PM_ERANGE, "k=%d not supported", k);
    } else {
        if (k != K) {
            return dispatch_hash<K + 1>(alphabet, k, u16, a, lds, blocks, st);
        }
        if (alphabet == 4)
            return u16 ? launch_hash<4, K, true>(a, lds, blocks, st) : launch_hash<4, K, false>(a, lds, blocks, st);
        if constexpr (K <= 7)
            return u16 ? launch_hash<20, K, true>(a, lds, blocks, st) : launch_hash<20, K, false>(a, lds, blocks, st);
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

// sizes the LDS (staged input, histogram slices) for the largest instance
// and launches one workgroup per (item, slice)
static int hash_launch(HashArgs &a, int A, int32_t items, int64_t x_max, int64_t nw_max, int t_max,
                       hipStream_t st)
{
    const bool u16 = x_max < 65536;
    const int lds_max = device_lds_bytes();
    a.seq_cap = nw_max * 4 <= 48 * 1024 ? (int)nw_max : 0;
    a.off_cap = (t_max + 1) * 4 <= 8 * 1024 ? t_max + 1 : 0;
    const int fixed = (a.seq_cap + a.off_cap) * 4;
    if (a.counts) {
        const int64_t need_words = u16 ? (a.nb + 1) / 2 : a.nb;
        int64_t budget = (lds_max - fixed) / 4;
        budget &= ~int64_t(3);
        if (budget < 1024) return fail(PM_ERANGE, "input too large for the LDS budget");
        int64_t hw = std::min<int64_t>(need_words, budget);
        // a whole-trial histogram that fits one workgroup but leaves it alone on
        // its CU goes into two balanced slices instead, so that two workgroups
        // share a CU and one's key pass overlaps the other's count write-out
        // (each slice recomputes the trial's keys; measured 11% faster on the
        // (18,6) workload's 128 KB histograms)
        const int64_t half = ((int64_t)lds_max / 2 - fixed) / 4;
        if (need_words <= budget && need_words > half && half >= 1024) hw = (need_words + 1) / 2;
        hw = (hw + 3) & ~int64_t(3);
        if (hw > budget) hw = budget;
        a.hist_words = (int)hw;
        a.slice_bins = (uint32_t)(u16 ? 2 * hw : hw);
        a.nslices = (int)((a.nb + a.slice_bins - 1) / a.slice_bins);
    } else {
        a.hist_words = 0;
        a.slice_bins = 0;
        a.nslices = 1;
    }
    const size_t lds = (size_t)a.hist_words * 4 + fixed;
    const int64_t blocks = (int64_t)items * a.nslices;
    if (blocks > 0x7fffffff) return fail(PM_ERANGE, "too many trials x slices");
    return dispatch_hash<1>(A, a.k, u16, a, lds, (int)blocks, st);
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
