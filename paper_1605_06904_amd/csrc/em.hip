// a7 - a10: OOPS EM refinement of every enriched bucket, and the final pick.
//
// Sec. 5.1 of the paper refines each enriched bucket with EM for a fixed
// number of iterations and keeps the model with the highest objective; it
// does not write the steps down.  The model here is the standard OOPS EM with
// a uniform start prior and a fixed background (see projmotif.h).
//
// Vector path: one workgroup (4 waves) per model.  The packed instance is
// staged in LDS; each wave owns whole sequences, so the per-sequence
// log-sum-exp is a wavefront reduction; the E-step reads the log-odds table
// from LDS; M-step counts go to per-wave LDS accumulators.
#include <math.h>

#include "pm_common.h"

namespace pm {

struct EmArgs {
    pm_inst one;                // the instance, when inst is NULL
    const pm_inst *inst;        // batch: instance table, or NULL
    const int32_t *item_inst;   // batch: instance of every trial item
    const pm_bucket *buckets;   // batch: the models' buckets (their items)
    const double *theta0;
    const double *bg;
    const int64_t *n_dev;
    double *theta_out;
    double *J;
    double *llr;
    int32_t *sites;
    int64_t B;
    int l, iters;
    int site_stride;  // sites row length (t, or the largest t of a batch)
    double beta;
    int model;        // PM_OOPS, PM_ZOOPS or PM_TCM
    double mix0;      // ZOOPS gamma or TCM lambda of theta0
    double *mix_out;  // [B] mixing parameter of the final E-step, or NULL
    int seq_cap;      // LDS words reserved for the packed input (0: read from global)
    int off_cap;      // LDS offsets reserved (0: read from global)
};

constexpr int kEmThreads = 256;
constexpr int kEmWaves = kEmThreads / 64;

template <typename T>
__device__ __forceinline__ T ninf();
template <>
__device__ __forceinline__ float ninf<float>() { return -INFINITY; }
template <>
__device__ __forceinline__ double ninf<double>() { return -INFINITY; }

__device__ __forceinline__ float ex(float v) { return expf(v); }
__device__ __forceinline__ double ex(double v) { return exp(v); }
__device__ __forceinline__ float lg1p(float v) { return log1pf(v); }
__device__ __forceinline__ double lg1p(double v) { return log1p(v); }

// ln(e^u + e^v), e^{-inf} = 0
template <typename T>
__device__ __forceinline__ T log_add(T u, T v)
{
    if (u == ninf<T>()) return v;
    if (v == ninf<T>()) return u;
    const T d = u - v;
    return (d > 0 ? u : v) + lg1p(ex(d > 0 ? -d : d));
}

template <typename V>
__device__ __forceinline__ V block_sum(V v, V *red)
{
    v = wave_sum(v);
    if (lane_id() == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    V r = red[0];
#pragma unroll
    for (int w = 1; w < kEmWaves; ++w) r += red[w];
    __syncthreads();
    return r;
}

__device__ __forceinline__ int64_t wave_min_i64(int64_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        int64_t u = __shfl_xor(v, o);
        v = u < v ? u : v;
    }
    return v;
}

template <typename T, int A>
__device__ __forceinline__ T score_at(const uint32_t *W, int64_t P, const T *Wt, int l)
{
    T s = 0;
    if (A == 4) {
        uint32_t hi, lo;
        dna_window(W, P, hi, lo);
        for (int p = 0; p < l; ++p) s += Wt[dna_at(hi, lo, p) * l + p];
    } else {
        for (int p = 0; p < l; ++p) s += Wt[prot_sym(W, P + p) * l + p];
    }
    return s;
}

template <typename T, int A>
__global__ void __launch_bounds__(kEmThreads) k_em_vec(const EmArgs a)
{
    const int64_t b = blockIdx.x;
    int64_t nvalid = a.n_dev ? *a.n_dev : a.B;
    if (nvalid > a.B) nvalid = a.B;
    if (b >= nvalid) return;

    __shared__ double th[A * 32];
    __shared__ T Wt[A * 32];
    __shared__ T acc[kEmWaves][A * 32];
    __shared__ double red[kEmWaves];
    __shared__ double colsum[32];
    __shared__ double ztot;
    extern __shared__ __align__(16) uint32_t dyn[];
    uint32_t *seq = dyn;
    int64_t *offs = reinterpret_cast<int64_t *>(dyn + ((a.seq_cap + 1) & ~1));

    const pm_inst I = a.inst ? a.inst[a.item_inst[a.buckets[b].trial]] : a.one;
    const int tid = threadIdx.x, wv = tid >> 6, lane = lane_id();
    const int l = a.l, t = I.t, AL = A * l;
    const double beta = a.beta;
    const int seq_words = a.seq_cap ? (int)(A == 4 ? (I.n_total + 15) / 16 + 4 : (I.n_total + 5) / 6 + 4) : 0;

    for (int i = tid; i < AL; i += kEmThreads) th[i] = a.theta0[b * AL + i];
    for (int i = tid; i < seq_words; i += kEmThreads) seq[i] = I.packed[i];
    if (a.off_cap)
        for (int i = tid; i <= t; i += kEmThreads) offs[i] = I.offsets[i];
    __syncthreads();
    const uint32_t *W = a.seq_cap ? seq : I.packed;
    const int64_t *O = a.off_cap ? offs : I.offsets;

    // mixing parameter of ZOOPS (gamma) or TCM (lambda); OOPS has none
    double mix = a.mix0;
    for (int it = 0; it <= a.iters; ++it) {
        const bool last = it == a.iters;
        const double lmix = log(mix), lnone = log1p(-mix);
        double pr = 0;
        for (int i = tid; i < AL; i += kEmThreads) {
            const int c = i / l;
            const double v = th[i];
            Wt[i] = (T)(log(v) - log(a.bg[c]));
            if (beta != 0) pr += a.bg[c] * log(v);
        }
        for (int i = tid; i < kEmWaves * A * 32; i += kEmThreads) (&acc[0][0])[i] = 0;
        pr = block_sum(pr, red);  // includes the barrier that publishes Wt

        double llr_w = 0;
        for (int i = wv; i < t; i += kEmWaves) {
            const int64_t s0 = O[i];
            const int64_t L = O[i + 1] - s0 - l + 1;
            if (a.model == PM_TCM) {
                // every window its own two-component mixture: one sweep gives
                // its log-likelihood term, its posterior and its counts
                const T lm = (T)lmix, ln0 = (T)lnone;
                double lsum = 0;
                T bv = ninf<T>();
                int64_t ba = 0;
                T *ac = acc[wv];
                for (int64_t x = lane; x < L; x += 64) {
                    const T s = score_at<T, A>(W, s0 + x, Wt, l);
                    const T v = lm + s;
                    const T li = log_add(ln0, v);
                    lsum += (double)li;
                    if (last) {
                        if (s > bv) {
                            bv = s;
                            ba = x;
                        }
                        continue;
                    }
                    const T z = v == ninf<T>() ? (T)0 : ex(v - li);
                    const int64_t P = s0 + x;
                    if (A == 4) {
                        uint32_t hi, lo;
                        dna_window(W, P, hi, lo);
                        for (int p = 0; p < l; ++p) atomicAdd(&ac[dna_at(hi, lo, p) * l + p], z);
                    } else {
                        for (int p = 0; p < l; ++p) atomicAdd(&ac[prot_sym(W, P + p) * l + p], z);
                    }
                }
                llr_w += wave_sum(lsum);
                if (last && a.sites) {
                    const T bm = wave_max(bv);
                    const int64_t cand = wave_min_i64(bv == bm ? ba : INT64_MAX);
                    // reported when that window's posterior is at least 1/2
                    const bool keep = (double)bm + lmix >= lnone;
                    if (lane == 0) a.sites[b * a.site_stride + i] = keep ? (int32_t)cand : -1;
                }
                continue;
            }
            // online log-sum-exp, one exponential per window; the exponentials
            // are in T, their running sum is FP64 in both precisions
            T mx = ninf<T>(), bv = ninf<T>();
            double sm = 0;
            int64_t ba = 0;
            for (int64_t x = lane; x < L; x += 64) {
                const T s = score_at<T, A>(W, s0 + x, Wt, l);
                const bool up = s > mx;
                const T e = ex(up ? mx - s : s - mx);
                sm = up ? sm * (double)e + 1.0 : (s > ninf<T>() ? sm + (double)e : sm);
                mx = up ? s : mx;
                if (last && s > bv) {
                    bv = s;
                    ba = x;
                }
            }
            const T M = wave_max(mx);
            const double part = mx > ninf<T>() ? sm * (double)ex(mx - M) : 0.0;
            const double Ssum = wave_sum(part);
            const double lse = (double)M + log(Ssum);
            // OOPS: LLR_i = LSE_i - ln L_i, Z = e^{s - LSE_i}.  ZOOPS: the
            // sequence holds no site with probability 1 - gamma, so
            // LLR_i = ln((1 - gamma) + gamma e^{LSE_i} / L_i) and
            // Z = gamma e^s / (L_i e^{LLR_i}); q_i = sum_a Z is its site mass
            double li, zoff, qi = 1.0;
            if (a.model == PM_ZOOPS) {
                const double lsite = lmix - log((double)L) + lse;
                li = log_add(lnone, lsite);
                zoff = lmix - log((double)L) - li;
                qi = exp(lsite - li);
            } else {
                li = lse - log((double)L);
                zoff = -lse;
            }
            llr_w += li;
            if (last) {
                if (a.sites) {
                    const T bm = wave_max(bv);
                    const int64_t cand = wave_min_i64(bv == bm ? ba : INT64_MAX);
                    if (lane == 0) a.sites[b * a.site_stride + i] = qi >= 0.5 ? (int32_t)cand : -1;
                }
            } else {
                T *ac = acc[wv];
                const T zo = (T)zoff;
                for (int64_t x = lane; x < L; x += 64) {
                    const T s = score_at<T, A>(W, s0 + x, Wt, l);
                    const T z = ex(s + zo);
                    const int64_t P = s0 + x;
                    if (A == 4) {
                        uint32_t hi, lo;
                        dna_window(W, P, hi, lo);
                        for (int p = 0; p < l; ++p) atomicAdd(&ac[dna_at(hi, lo, p) * l + p], z);
                    } else {
                        for (int p = 0; p < l; ++p) atomicAdd(&ac[prot_sym(W, P + p) * l + p], z);
                    }
                }
            }
        }
        // every lane of a wave holds the same llr_w; count each wave once
        const double llr = block_sum(lane == 0 ? llr_w : 0.0, red);
        if (tid == 0) {
            a.J[b * (a.iters + 1) + it] = llr + beta * pr;
            if (a.llr) a.llr[b * (a.iters + 1) + it] = llr;
        }
        if (!last) {
            // counts of the four waves, summed in FP64
            for (int i = tid; i < AL; i += kEmThreads) {
                double cs = 0;
#pragma unroll
                for (int w = 0; w < kEmWaves; ++w) cs += (double)acc[w][i];
                th[i] = cs;
            }
            __syncthreads();
            // theta' = (counts + beta*bg) / (t + beta); every column's counts sum
            // to t, so dividing by the column's own total is the same update and
            // keeps each column exactly on the simplex under rounding
            for (int p = tid; p < l; p += kEmThreads) {
                double tot = 0;
                for (int c = 0; c < A; ++c) tot += th[c * l + p];
                colsum[p] = tot + beta;
                if (p == 0) ztot = tot;
            }
            __syncthreads();
            for (int i = tid; i < AL; i += kEmThreads) th[i] = (th[i] + beta * a.bg[i / l]) / colsum[i % l];
            // the mixing parameter's update: the posterior mass (every
            // column's counts total it) over t sequences (ZOOPS) or x windows
            // (TCM), capped at 1 against rounding
            if (a.model == PM_ZOOPS) mix = fmin(1.0, ztot / (double)t);
            else if (a.model == PM_TCM) mix = fmin(1.0, ztot / (double)I.x);
            __syncthreads();
        }
    }
    for (int i = tid; i < AL; i += kEmThreads) a.theta_out[b * AL + i] = th[i];
    if (tid == 0 && a.mix_out) a.mix_out[b] = mix;
}

template <typename T, int A>
static int launch_em(const EmArgs &a, size_t lds, hipStream_t st)
{
    hipLaunchKernelGGL((k_em_vec<T, A>), dim3((unsigned)a.B), dim3(kEmThreads), lds, st, a);
    PM_LAUNCHED();
    return PM_OK;
}

// ---------------------------------------------------------------- a10
// one workgroup per instance (inst != NULL: a batch, whose buckets ascend by
// item) or a single workgroup over all buckets
constexpr int kBestThreads = 1024;
constexpr int kBestUnroll = 8;  // final objectives in flight per thread

__global__ void __launch_bounds__(kBestThreads) k_best(const double *J, int64_t B, const int64_t *n_dev, int iters,
                                                       const double *theta, int A, int l, int64_t *best_out,
                                                       char *cons, const pm_inst *inst, const pm_bucket *buckets)
{
    __shared__ double rv[kBestThreads / kWave];
    __shared__ int64_t ri[kBestThreads / kWave];
    __shared__ int64_t best_s;
    int64_t nvalid = n_dev ? *n_dev : B;
    if (nvalid > B) nvalid = B;
    int64_t lo_b = 0, hi_b = nvalid;
    if (inst) {
        const int p = blockIdx.x;
        int64_t r[2];
        for (int side = 0; side < 2; ++side) {
            const int64_t item = (int64_t)inst[p].first_item + (side ? inst[p].m : 0);
            int64_t lo = 0, hi = nvalid;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if ((int64_t)buckets[mid].trial < item) lo = mid + 1;
                else hi = mid;
            }
            r[side] = lo;
        }
        lo_b = r[0];
        hi_b = r[1];
        best_out += p;
        if (cons) cons += (int64_t)p * (l + 1);
    }
    double bv = -INFINITY;
    int64_t bi = INT64_MAX;
    // each thread takes its buckets in ascending order, several loads at a time
    const int64_t stride = (int64_t)iters + 1;
    for (int64_t b0 = lo_b + threadIdx.x; b0 < hi_b; b0 += (int64_t)kBestUnroll * kBestThreads) {
        double v[kBestUnroll];
#pragma unroll
        for (int u = 0; u < kBestUnroll; ++u) {
            const int64_t b = b0 + (int64_t)u * kBestThreads;
            v[u] = b < hi_b ? J[b * stride + iters] : NAN;
        }
#pragma unroll
        for (int u = 0; u < kBestUnroll; ++u) {
            if (v[u] == v[u] && (bi == INT64_MAX || v[u] > bv)) {
                bv = v[u];
                bi = b0 + (int64_t)u * kBestThreads;
            }
        }
    }
    // (value, index): larger value wins, then smaller index
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(bv, o);
        const int64_t oi = __shfl_xor(bi, o);
        if (oi != INT64_MAX && (bi == INT64_MAX || ov > bv || (ov == bv && oi < bi))) {
            bv = ov;
            bi = oi;
        }
    }
    if (lane_id() == 0) {
        rv[threadIdx.x >> 6] = bv;
        ri[threadIdx.x >> 6] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = rv[0];
        int64_t i = ri[0];
        for (int w = 1; w < kBestThreads / kWave; ++w)
            if (ri[w] != INT64_MAX && (i == INT64_MAX || rv[w] > v || (rv[w] == v && ri[w] < i))) {
                v = rv[w];
                i = ri[w];
            }
        best_s = i == INT64_MAX ? -1 : i;
        best_out[0] = best_s;
    }
    __syncthreads();
    const int64_t bb = best_s;
    if (!cons) return;
    const char *letters = A == 4 ? "ACTG" : "ARNDCQEGHILKMFPSTWYV";
    if ((int)threadIdx.x < l) {
        char ch = 0;
        if (bb >= 0) {
            const double *th = theta + bb * A * l;
            int bc = 0;
            for (int c = 1; c < A; ++c)
                if (th[c * l + threadIdx.x] > th[bc * l + threadIdx.x]) bc = c;
            ch = letters[bc];
        }
        cons[threadIdx.x] = ch;
    }
    if (threadIdx.x == 0) cons[l] = 0;
}

}  // namespace pm

using namespace pm;

static int check_em_args(int A, int64_t B, int32_t iters, double beta, int32_t precision, const double *theta0,
                         const double *bg, const double *theta_out, const double *J_out)
{
    if (B < 0 || iters < 0 || beta < 0) return fail(PM_EINVAL, "need B >= 0, iters >= 0, beta >= 0");
    if (precision != PM_FP64 && precision != PM_FP32 && precision != PM_F16X2 && precision != PM_F16)
        return fail(PM_EINVAL, "unknown precision %d", precision);
    if (precision == PM_F16X2 && A != 4) return fail(PM_EINVAL, "PM_F16X2 is for DNA");
    if (B > 0x7fffffff) return fail(PM_ERANGE, "B above 2^31 - 1");
    if (B > 0 && (!theta0 || !bg || !theta_out || !J_out)) return fail(PM_EINVAL, "NULL buffer");
    return PM_OK;
}

static int vec_launch(EmArgs &a, int A, int32_t precision, int64_t nw_max, int t_max, hipStream_t st)
{
    a.seq_cap = nw_max * 4 <= 48 * 1024 ? (int)nw_max : 0;
    a.off_cap = (t_max + 1) * 8 <= 8 * 1024 ? t_max + 1 : 0;
    const size_t lds = ((a.seq_cap + 1) & ~1) * 4 + (size_t)a.off_cap * 8;
    if (A == 4)
        return precision == PM_FP64 ? launch_em<double, 4>(a, lds, st) : launch_em<float, 4>(a, lds, st);
    return precision == PM_FP64 ? launch_em<double, 20>(a, lds, st) : launch_em<float, 20>(a, lds, st);
}

extern "C" size_t pm_em_workspace(const pm_seqs *S, int32_t l, int32_t precision)
{
    clear_error();
    if (check_seqs(S, l) != PM_OK) return 0;
    if (S->alphabet != 4 || (precision != PM_F16X2 && precision != PM_F16)) return 0;
    return em_tables_workspace(S, l);
}

extern "C" int em_refine(const pm_seqs *S, int32_t l, const double *theta0, const double *bg, int64_t B,
                         const int64_t *n_dev, int32_t iters, double beta, int32_t precision,
                         double *theta_out, double *J_out, double *llr_out, int32_t *sites_out,
                         void *ws, size_t ws_bytes, void *stream)
{
    clear_error();
    int rc = check_seqs(S, l);
    if (rc) return rc;
    if ((rc = check_em_args(S->alphabet, B, iters, beta, precision, theta0, bg, theta_out, J_out))) return rc;
    if (B == 0) return PM_OK;
    hipStream_t st = as_stream(stream);
    if (precision == PM_F16 && S->alphabet == 20)
        return em_refine_prot(S, l, theta0, bg, B, n_dev, iters, beta, theta_out, J_out, llr_out, sites_out, st);
    if (precision == PM_F16X2 || precision == PM_F16)
        return em_refine_mfma(S, l, theta0, bg, B, n_dev, iters, beta, theta_out, J_out, llr_out, sites_out, ws,
                              ws_bytes, precision == PM_F16X2, st);
    EmArgs a{};
    a.one = inst_of(S, l);
    a.theta0 = theta0;
    a.bg = bg;
    a.n_dev = n_dev;
    a.theta_out = theta_out;
    a.J = J_out;
    a.llr = llr_out;
    a.sites = sites_out;
    a.B = B;
    a.l = l;
    a.iters = iters;
    a.site_stride = S->t;
    a.beta = beta;
    return vec_launch(a, S->alphabet, precision, pm_packed_words(S->alphabet, S->n_total), S->t, st);
}

extern "C" int em_refine_model(const pm_seqs *S, int32_t l, int32_t model, double mix0, const double *theta0,
                               const double *bg, int64_t B, const int64_t *n_dev, int32_t iters, double beta,
                               int32_t precision, double *theta_out, double *mix_out, double *J_out,
                               double *llr_out, int32_t *sites_out, void *stream)
{
    clear_error();
    if (model == PM_OOPS)
        return em_refine(S, l, theta0, bg, B, n_dev, iters, beta, precision, theta_out, J_out, llr_out, sites_out,
                         nullptr, 0, stream);
    int rc = check_seqs(S, l);
    if (rc) return rc;
    if (model != PM_ZOOPS && model != PM_TCM) return fail(PM_EINVAL, "unknown sequence model %d", model);
    if (!(mix0 > 0.0 && mix0 <= 1.0)) return fail(PM_EINVAL, "the mixing parameter must lie in (0, 1] (%g)", mix0);
    if (precision != PM_FP64 && precision != PM_FP32)
        return fail(PM_EINVAL, "ZOOPS and TCM run in PM_FP64 or PM_FP32 (precision %d)", precision);
    if ((rc = check_em_args(S->alphabet, B, iters, beta, precision, theta0, bg, theta_out, J_out))) return rc;
    if (B == 0) return PM_OK;
    EmArgs a{};
    a.one = inst_of(S, l);
    a.theta0 = theta0;
    a.bg = bg;
    a.n_dev = n_dev;
    a.theta_out = theta_out;
    a.J = J_out;
    a.llr = llr_out;
    a.sites = sites_out;
    a.B = B;
    a.l = l;
    a.iters = iters;
    a.site_stride = S->t;
    a.beta = beta;
    a.model = model;
    a.mix0 = mix0;
    a.mix_out = mix_out;
    return vec_launch(a, S->alphabet, precision, pm_packed_words(S->alphabet, S->n_total), S->t, as_stream(stream));
}

extern "C" size_t pm_em_batch_workspace(const pm_batch *B, int32_t precision)
{
    clear_error();
    BatchInfo info;
    if (check_batch(B, &info) != PM_OK) return 0;
    const bool mfma = B->alphabet == 4 && (precision == PM_F16X2 || precision == PM_F16);
    return mfma ? em_batch_workspace(B, true) : 0;
}

extern "C" int em_autotune(const pm_seqs *S, int32_t l, const double *theta0, const double *bg, int64_t B,
                           int32_t iters, double beta, int32_t precision, double *theta_out, double *J_out,
                           void *ws, size_t ws_bytes, int32_t *choice_out, void *stream)
{
    clear_error();
    int rc = check_seqs(S, l);
    if (rc) return rc;
    if (precision != PM_F16X2 && precision != PM_F16) return fail(PM_EINVAL, "only the matrix-core forms are tuned");
    if ((rc = check_em_args(S->alphabet, B, iters, beta, precision, theta0, bg, theta_out, J_out))) return rc;
    if (B < 1) return fail(PM_EINVAL, "need B >= 1 models to time");
    if (S->alphabet != 4) return fail(PM_EINVAL, "the tuned tile shapes are those of the DNA matrix-core form");
    return em_autotune_mfma(S, l, theta0, bg, B, iters, beta, precision == PM_F16X2, theta_out, J_out, ws, ws_bytes,
                            choice_out, as_stream(stream));
}

extern "C" int em_tuning(int32_t l, int32_t precision)
{
    clear_error();
    if (l < 1 || l > 32 || (precision != PM_F16X2 && precision != PM_F16)) return fail(PM_EINVAL, "bad l/precision");
    return em_tuned_shape(l, precision == PM_F16X2);
}

extern "C" int em_set_tuning(int32_t l, int32_t precision, int32_t shape)
{
    clear_error();
    if (l < 1 || l > 32 || (precision != PM_F16X2 && precision != PM_F16)) return fail(PM_EINVAL, "bad l/precision");
    return em_record_shape(l, precision == PM_F16X2, shape);
}

extern "C" int em_refine_batch(const pm_batch *Bt, const pm_bucket *buckets, const double *theta0, const double *bg,
                               int64_t B, const int64_t *n_dev, int32_t iters, double beta, int32_t precision,
                               double *theta_out, double *J_out, double *llr_out, int32_t *sites_out, void *ws,
                               size_t ws_bytes, void *stream)
{
    clear_error();
    BatchInfo info;
    int rc = check_batch(Bt, &info);
    if (rc) return rc;
    if ((rc = check_em_args(Bt->alphabet, B, iters, beta, precision, theta0, bg, theta_out, J_out))) return rc;
    if (B == 0) return PM_OK;
    if (!buckets) return fail(PM_EINVAL, "buckets are NULL");
    hipStream_t st = as_stream(stream);
    if (precision == PM_F16 && Bt->alphabet == 20)
        return fail(PM_EINVAL, "the protein matrix-core form runs on single instances (em_refine)");
    if (precision == PM_F16X2 || precision == PM_F16) {
        const size_t need = em_batch_workspace(Bt, true);
        if (!ws || ws_bytes < need) return fail(PM_EINVAL, "workspace of %zu bytes, need %zu", ws ? ws_bytes : 0, need);
        if (((uintptr_t)ws & 255) != 0) return fail(PM_EINVAL, "workspace must be 256-byte aligned");
        return em_refine_mfma_batch(Bt, info.nw_max, info.t_max, buckets, theta0, bg, B, n_dev, iters, beta,
                                    theta_out, J_out, llr_out, sites_out, ws, precision == PM_F16X2, st);
    }
    EmArgs a{};
    a.inst = Bt->inst;
    a.item_inst = Bt->item_inst;
    a.buckets = buckets;
    a.theta0 = theta0;
    a.bg = bg;
    a.n_dev = n_dev;
    a.theta_out = theta_out;
    a.J = J_out;
    a.llr = llr_out;
    a.sites = sites_out;
    a.B = B;
    a.l = Bt->l;
    a.iters = iters;
    a.site_stride = info.t_max;
    a.beta = beta;
    return vec_launch(a, Bt->alphabet, precision, info.nw_max, info.t_max, st);
}

extern "C" int em_best(const double *J, int64_t B, const int64_t *n_dev, int32_t iters, const double *theta,
                       int32_t alphabet, int32_t l, int64_t *best_out, char *consensus_out, void *stream)
{
    clear_error();
    if (alphabet != 4 && alphabet != 20) return fail(PM_EINVAL, "alphabet must be 4 or 20");
    if (l < 1 || l > 32 || B < 0 || iters < 0) return fail(PM_EINVAL, "bad sizes");
    if (!best_out || (B > 0 && (!J || !theta))) return fail(PM_EINVAL, "NULL buffer");
    hipLaunchKernelGGL(k_best, dim3(1), dim3(kBestThreads), 0, as_stream(stream), J, B, n_dev, iters, theta,
                       alphabet, l, best_out, consensus_out, nullptr, nullptr);
    PM_LAUNCHED();
    return PM_OK;
}

extern "C" int em_best_batch(const pm_batch *Bt, const pm_bucket *buckets, const double *J, int64_t B,
                             const int64_t *n_dev, int32_t iters, const double *theta, int64_t *best_out,
                             char *consensus_out, void *stream)
{
    clear_error();
    int rc = check_batch(Bt, nullptr);
    if (rc) return rc;
    if (B < 0 || iters < 0) return fail(PM_EINVAL, "bad sizes");
    if (!best_out || (B > 0 && (!J || !theta || !buckets))) return fail(PM_EINVAL, "NULL buffer");
    hipLaunchKernelGGL(k_best, dim3(Bt->P), dim3(kBestThreads), 0, as_stream(stream), J, B, n_dev, iters, theta,
                       Bt->alphabet, Bt->l, best_out, consensus_out, Bt->inst, buckets);
    PM_LAUNCHED();
    return PM_OK;
}
