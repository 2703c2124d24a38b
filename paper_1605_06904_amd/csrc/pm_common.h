// Shared device helpers and host error plumbing of libprojmotif (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "projmotif.h"

namespace pm {

// ---------------------------------------------------------------- host side
int fail(int code, const char *fmt, ...);
void clear_error();
int device_lds_bytes();  // max dynamic LDS per workgroup on the current device
hipStream_t as_stream(void *s);

#define PM_TRY(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return ::pm::fail(PM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define PM_LAUNCHED()                                                                         \
    do {                                                                                      \
        hipError_t e_ = hipGetLastError();                                                    \
        if (e_ != hipSuccess)                                                                 \
            return ::pm::fail(PM_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e_)); \
    } while (0)

static inline int64_t ipow(int64_t a, int k)
{
    int64_t r = 1;
    for (int i = 0; i < k; ++i) r *= a;
    return r;
}

// windows of the instance for motif length l
static inline int64_t num_windows(const pm_seqs *S, int l)
{
    return S->n_total - (int64_t)S->t * (l - 1);
}

int check_seqs(const pm_seqs *S, int l);

// a single instance seen as a one-instance batch entry (key_base 0, item 0)
pm_inst inst_of(const pm_seqs *S, int l);

// launch sizes of a batch: the largest instance in each respect
struct BatchInfo {
    int t_max;
    int64_t nw_max;      // packed words
    int64_t x_max;       // windows
    int64_t keys_total;  // key slots over all items
};
int check_batch(const pm_batch *B, BatchInfo *info);

// exclusive scan of n per-entry (bucket, member) totals into bases; writes the
// grand totals to n_out and PM_STATUS_CAPACITY when they exceed the capacities.
// With `heavy` set, also lists in order the entries with more than heavy_above
// buckets, and their number in n_heavy.  With parts > 1 the totals of entry j
// are the sums of ne/ms[j * parts .. j * parts + parts - 1], also written to
// ne_sum/ms_sum.
struct TotScan {
    const int64_t *ne, *ms;
    int64_t *bb, *mb;
    int64_t n, cap_b, cap_m;
    int64_t *n_out;
    uint32_t *status;
    int32_t *heavy;
    int64_t *n_heavy;
    int64_t heavy_above;
    int parts;
    int64_t *ne_sum, *ms_sum;
    int64_t *max_heavy;  // with `heavy`: the most buckets of a heavy entry (or NULL)
};
int launch_tot_scan(const TotScan &a, hipStream_t st);

// projection_hash_select: the pieces of bucket_select's workspace that its
// hash pass writes (passing-key bitmap, per-trial passing bins and members),
// with the totals zeroed on the stream; then the selection from them, the
// counting pass skipped.  The workspace is bucket_select's.
struct SelCounted {
    uint64_t *bits;
    int64_t *ne, *ms;
    int64_t nwb;
};
int check_select_ws(int A, int k, int32_t items, const uint32_t *keys, const uint32_t *counts,
                    const int64_t *n_out, void *ws, size_t ws_bytes, pm_bucket *buckets, int64_t cap_buckets,
                    uint32_t *members, int64_t cap_members);
int select_counted_prepare(void *ws, int32_t m, int A, int k, SelCounted *out, hipStream_t st);
int select_counted(const pm_inst &one, const pm_inst *inst, const int32_t *item_inst, int A, int k,
                   const uint32_t *keys, const uint32_t *counts, int32_t m, uint32_t s, pm_bucket *buckets,
                   int64_t cap_buckets, uint32_t *members, int64_t cap_members, int64_t *n_out, void *ws,
                   uint32_t *status, int64_t x_max, hipStream_t st);

int em_refine_mfma(const pm_seqs *S, int32_t l, const double *theta0, const double *bg, int64_t B,
                   const int64_t *n_dev, int32_t iters, double beta, double *theta_out, double *J_out,
                   double *llr_out, int32_t *sites_out, void *ws, size_t ws_bytes, bool split, hipStream_t st);
size_t em_tables_workspace(const pm_seqs *S, int32_t l);
int em_refine_mfma_batch(const pm_batch *Bt, int64_t nw_max, int t_max, const pm_bucket *buckets,
                         const double *theta0, const double *bg, int64_t B, const int64_t *n_dev, int32_t iters,
                         double beta, double *theta_out, double *J_out, double *llr_out, int32_t *sites_out,
                         void *ws, bool split, hipStream_t st);
size_t em_batch_workspace(const pm_batch *Bt, bool tables);
int em_autotune_mfma(const pm_seqs *S, int32_t l, const double *theta0, const double *bg, int64_t B, int32_t iters,
                     double beta, bool split, double *theta_out, double *J_out, void *ws, size_t ws_bytes,
                     int32_t *choice, hipStream_t st);
int em_tuned_shape(int32_t l, bool split);
int em_record_shape(int32_t l, bool split, int32_t shape);
int em_refine_prot(const pm_seqs *S, int32_t l, const double *theta0, const double *bg, int64_t B,
                   const int64_t *n_dev, int32_t iters, double beta, double *theta_out, double *J_out,
                   double *llr_out, int32_t *sites_out, hipStream_t st);

// ---------------------------------------------------------------- device side
constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Symbol g of a DNA sequence packed 16 per word, first symbol in bits 31..30.
__device__ __forceinline__ uint32_t dna_sym(const uint32_t *w, int64_t g)
{
    return (w[g >> 4] >> (30 - ((uint32_t)(g & 15) << 1))) & 3u;
}

// 32 consecutive DNA symbols starting at P: symbols P..P+15 in `hi`,
// P+16..P+31 in `lo`, each MSB-first.  Reads words P/16 .. P/16+2.
__device__ __forceinline__ void dna_window(const uint32_t *w, int64_t P, uint32_t &hi, uint32_t &lo)
{
    const int64_t wi = P >> 4;
    const uint32_t r = (uint32_t)(P & 15) << 1;
    const uint64_t a = ((uint64_t)w[wi] << 32) | w[wi + 1];
    const uint64_t b = ((uint64_t)w[wi + 1] << 32) | w[wi + 2];
    hi = (uint32_t)(a >> (32 - r));
    lo = (uint32_t)(b >> (32 - r));
}

// Symbol p (0..31) of a window fetched by dna_window.
__device__ __forceinline__ uint32_t dna_at(uint32_t hi, uint32_t lo, int p)
{
    const uint32_t src = p < 16 ? hi : lo;
    return (src >> (30 - ((p & 15) << 1))) & 3u;
}

// floor(g / 6) for 0 <= g < 2^32.
__device__ __forceinline__ uint32_t div6(uint32_t g)
{
    return (uint32_t)(((uint64_t)g * 0xAAAAAAABull) >> 34);
}

// Symbol g of a protein sequence packed 6 per word (5 bits each), first
// symbol in bits 31..27.
__device__ __forceinline__ uint32_t prot_sym(const uint32_t *w, int64_t g)
{
    const uint32_t q = div6((uint32_t)g);
    const uint32_t r = (uint32_t)g - 6u * q;
    return (w[q] >> (27 - 5 * r)) & 31u;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T u = __shfl_xor(v, o);
        v = u > v ? u : v;
    }
    return v;
}

// inclusive prefix sum over the 64 lanes (all lanes active)
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t n = __shfl_up(v, o);
        if (lane >= o) v += n;
    }
    return v;
}

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }


}  // namespace pm
