// Device pieces shared by the projection kernels of libprojmotif (gfx950):
// the launch arguments of a trial item, the LDS staging of an instance's
// packed input, and the projected key of every window (Sec. 5 projection,
// Sec. 6 base-|Sigma| integer, most significant symbol first).
#pragma once

#include "pm_common.h"

namespace pm {

struct HashArgs {
    pm_inst one;               // the instance, when inst is NULL
    const pm_inst *inst;       // batch: instance table, or NULL
    const int32_t *item_inst;  // batch: instance of every trial item
    const uint32_t *masks;
    uint32_t *keys;
    uint32_t *counts;
    uint32_t *status;
    int64_t nb;          // |Sigma|^k
    int A, l, k;         // alphabet size, motif length, projection size
    int nslices;         // key-range slices per trial
    uint32_t slice_bins; // bins per slice (multiple of 4)
    int hist_words;      // LDS words of histogram
    int seq_cap;         // LDS words reserved for the input (0: read from global): DNA the packed
                         // words, protein one byte per symbol (unpacked on staging)
    int off_cap;         // LDS window starts reserved, t + 1 (0: read offsets from global)
    // projection_hash_select: with the counts, the selection's passing-key
    // bitmap (words of 64 bins in lane-major bit order: bit 16q + i of the
    // word of bins 64w .. 64w+63 is bin 64w + 4i + q) and per item the number
    // of passing bins and their members, added up over the item's slices
    // (zeroed before the launch); slices are then whole 256-bin groups.  NULL
    // in projection_hash.
    uint64_t *sel_bits;        // [items][sel_nwb]
    int64_t *sel_ne, *sel_ms;  // [items]
    int64_t sel_nwb;
    uint32_t sel_smin;         // a bin passes with at least this many l-mers
};

constexpr int kHashThreads = 1024;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// The instance of trial item j, with its packed input (and the window number
// of every sequence start) staged in LDS when the launch reserved room.
struct Staged {
    pm_inst I;
    const uint32_t *seq;  // LDS copy (seq_cap; protein: bytes) or the global packed words
    const int32_t *wst;   // LDS window starts, when off_cap
};

template <int A>
__device__ __forceinline__ Staged stage_input(const HashArgs &a, int j, uint32_t *seq, int32_t *wst)
{
    const pm_inst I = a.inst ? a.inst[a.item_inst[j]] : a.one;
    const int seq_words = a.seq_cap ? (int)(A == 4 ? (I.n_total + 15) / 16 + 4 : (I.n_total + 5) / 6 + 4) : 0;
    if (A == 4) {
        for (int i = threadIdx.x; i < seq_words; i += kHashThreads) seq[i] = I.packed[i];
    } else {
        // protein: one byte per symbol, so that a key reads each projected
        // symbol with one LDS byte load instead of a division by six
        uint8_t *sb = reinterpret_cast<uint8_t *>(seq);
        for (int i = threadIdx.x; i < seq_words; i += kHashThreads) {
            const uint32_t v = I.packed[i];
#pragma unroll
            for (int q = 0; q < 6; ++q) sb[6 * i + q] = (uint8_t)((v >> (27 - 5 * q)) & 31u);
        }
    }
    if (a.off_cap)
        for (int i = threadIdx.x; i <= I.t; i += kHashThreads) wst[i] = (int32_t)(I.offsets[i] - (int64_t)i * (a.l - 1));
    return Staged{I, a.seq_cap ? seq : I.packed, wst};
}

// kept positions, ascending: the shift of each kept position's 2-bit field in
// the 64-bit window (DNA), or the position itself (protein)
template <int A, int K>
__device__ __forceinline__ void kept_positions(uint32_t mask, int (&pos)[K])
{
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const int p = __builtin_ctz(mask);
        pos[q] = A == 4 ? 62 - 2 * p : p;
        mask &= mask - 1;
    }
}

// fn(w, key) for every window w = tid, tid + kHashThreads, ... of the instance
template <int A, int K, typename F>
__device__ __forceinline__ void for_each_key(const HashArgs &a, const Staged &st, const int (&pos)[K], F &&fn)
{
    const int64_t x = st.I.x;
    if (a.seq_cap && a.off_cap) {
        // staged input: every read below is an LDS read, all indices 32-bit
        // (n_total < 2^31)
        const uint32_t *seq = st.seq;
        const int32_t *wst = st.wst;
        const uint32_t x32 = (uint32_t)x, lm1 = (uint32_t)(a.l - 1);
        int i = 0;
        for (uint32_t w = threadIdx.x; w < x32; w += kHashThreads) {
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
                const uint8_t *sb = reinterpret_cast<const uint8_t *>(seq);
#pragma unroll
                for (int q = 0; q < K; ++q) key = key * 20u + sb[P + (uint32_t)pos[q]];
            }
            fn((int64_t)w, key);
        }
    } else {
        // large instances: packed input and offsets read from global memory
        const uint32_t *W = st.seq;
        const int64_t *O = st.I.offsets;
        const int64_t lm1 = a.l - 1;
        int i = 0;
        for (int64_t w = threadIdx.x; w < x; w += kHashThreads) {
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
            fn(w, key);
        }
    }
}

__device__ __forceinline__ bool mask_ok(const HashArgs &a, uint32_t mask)
{
    const uint32_t lmask = a.l == 32 ? 0xffffffffu : ((1u << a.l) - 1u);
    return __popc(mask) == a.k && !(mask & ~lmask);
}

// LDS words that stage an instance of nw packed words: the words themselves
// (DNA) or one byte per symbol (protein, six per word)
__host__ __device__ inline int64_t staged_words(int A, int64_t nw) { return A == 4 ? nw : (6 * nw + 3) / 4; }

// The key of window w (w < x), with i the sequence index of an earlier
// window of the caller (0 at the start; advanced here).  Same arithmetic as
// for_each_key, for loops whose trip count must be the same in every thread.
template <int A, int K>
__device__ __forceinline__ uint32_t window_key(const HashArgs &a, const Staged &st, const int (&pos)[K], int64_t w,
                                               int &i)
{
    uint32_t key = 0;
    if (a.seq_cap && a.off_cap) {
        const uint32_t *seq = st.seq;
        const int32_t *wst = st.wst;
        while ((int32_t)w >= wst[i + 1]) ++i;
        const uint32_t P = (uint32_t)w + (uint32_t)i * (uint32_t)(a.l - 1);
        if (A == 4) {
            const uint32_t wi = P >> 4, r = (P & 15u) << 1;
            const uint32_t w0 = seq[wi], w1 = seq[wi + 1], w2 = seq[wi + 2];
            const uint32_t hi = (uint32_t)((((uint64_t)w0 << 32) | w1) >> (32 - r));
            const uint32_t lo = (uint32_t)((((uint64_t)w1 << 32) | w2) >> (32 - r));
            const uint64_t win = ((uint64_t)hi << 32) | lo;
#pragma unroll
            for (int q = 0; q < K; ++q) key = (key << 2) | ((uint32_t)(win >> pos[q]) & 3u);
        } else {
            const uint8_t *sb = reinterpret_cast<const uint8_t *>(seq);
#pragma unroll
            for (int q = 0; q < K; ++q) key = key * 20u + sb[P + (uint32_t)pos[q]];
        }
    } else {
        const int64_t *O = st.I.offsets;
        const int64_t lm1 = a.l - 1;
        while (w >= O[i + 1] - (int64_t)(i + 1) * lm1) ++i;
        const int64_t P = w + (int64_t)i * lm1;
        if (A == 4) {
            uint32_t hi, lo;
            dna_window(st.seq, P, hi, lo);
            const uint64_t win = ((uint64_t)hi << 32) | lo;
#pragma unroll
            for (int q = 0; q < K; ++q) key = (key << 2) | ((uint32_t)(win >> pos[q]) & 3u);
        } else {
#pragma unroll
            for (int q = 0; q < K; ++q) key = key * 20u + prot_sym(st.seq, P + pos[q]);
        }
    }
    return key;
}

// ---- the sorted selection (sortsel.hip), for key spaces beyond LDS
// histograms: DNA k from kSortKMinDna to 16, protein k from kSortKMinProt to 7
constexpr int kSortKMinDna = 8;
constexpr int kSortKMinProt = 4;
int hsort_check_k(int A, int k);
size_t hsort_workspace(int A, int l, int k, int32_t items, int64_t x_max, int64_t nw_max, int t_max);
int hsort_run(HashArgs &a, int A, int32_t items, int64_t x_max, int64_t nw_max, int t_max, uint32_t s,
              pm_bucket *buckets, int64_t cap_b, uint32_t *members, int64_t cap_m, int64_t *n_out, void *ws,
              size_t ws_bytes, hipStream_t st);

}  // namespace pm
