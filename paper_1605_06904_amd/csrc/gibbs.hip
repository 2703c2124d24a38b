// Gibbs site sampling as the local optimiser of a bucket, in place of EM.
//
// Sec. 1 and Sec. 3 of the paper name Gibbs sampling beside EM as the local
// search that PROJECTION seeds; the sampler is the site sampler of Lawrence
// et al. (cited there).  Per model: start from the best start of every
// sequence under the bucket's theta0; a sweep visits the sequences in order
// and redraws each one's start from the motif model of the other t-1 sites
// (pseudocounts beta * bg); the alignment of largest log-odds score F over
// the start and every sweep is the answer.  Random numbers come from
// Philox4x64-10 (Salmon et al., SC'11) keyed by the seed, one block per
// (sweep, sequence, model), so any model's chain is reproducible on its own.
//
// One wave per model, four models (one instance) per workgroup; the packed
// instance is staged in LDS once for the four.  A draw scores the sequence's
// starts in contiguous chunks per lane (lane order = start order), so a wave
// scan of the lanes' weight sums gives every lane's running sum and the lane
// holding the drawn start walks its chunk once more to find it.  All
// arithmetic is FP64.
#include <math.h>

#include "pm_common.h"

namespace pm {

constexpr int kGibbsWaves = 4;
constexpr int kGibbsThreads = kGibbsWaves * kWave;
constexpr int kGibbsMaxT = 512;

struct GibbsArgs {
    pm_inst one;
    const double *theta0;
    const double *bg;
    const int64_t *n_dev;
    double *theta_out;
    double *F;
    int32_t *sites;
    int64_t B;
    int l, A, sweeps;
    double beta;
    uint64_t seed;
    int seq_cap;  // LDS words of the packed input (0: global)
    int off_cap;  // LDS offsets (0: global)
};

__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t lo0 = M0 * c[0], hi0 = __umul64hi(M0, c[0]);
        const uint64_t lo1 = M1 * c[2], hi1 = __umul64hi(M1, c[2]);
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
}

// uniform in [0, 1) with 53 random bits for (sweep, sequence, model)
__device__ __forceinline__ double gibbs_uniform(uint64_t seed, int sweep, int i, int64_t model)
{
    uint64_t c[4] = {(uint64_t)sweep, (uint64_t)i, (uint64_t)model, 0};
    philox4x64_10(c, seed, 0);
    return (double)(c[0] >> 11) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ int sym_at(int A, const uint32_t *W, int64_t g)
{
    return A == 4 ? (int)dna_sym(W, g) : (int)prot_sym(W, g);
}

// score of start a of the sequence beginning at symbol s0 under table Wt
__device__ __forceinline__ double start_score(int A, const uint32_t *W, int64_t s0, int64_t a, const double *Wt, int l)
{
    double v = 0;
    for (int p = 0; p < l; ++p) v += Wt[sym_at(A, W, s0 + a + p) * l + p];
    return v;
}

// F = sum n ln(theta / bg) over entries with n > 0, theta = (n + beta bg)/(t + beta)
__device__ __forceinline__ double alignment_F(const int32_t *n, const double *bg, int A, int l, int t, double beta)
{
    double f = 0;
    for (int e = lane_id(); e < A * l; e += kWave) {
        const int c = e / l;
        if (n[e] > 0) f += (double)n[e] * log(((double)n[e] + beta * bg[c]) / ((double)t + beta) / bg[c]);
    }
    return wave_sum(f);
}

// (value, index) with the larger value, the smaller index on ties
__device__ __forceinline__ void wave_argmax(double &v, int64_t &ix)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(v, o);
        const int64_t oi = __shfl_xor(ix, o);
        if (ov > v || (ov == v && oi < ix)) {
            v = ov;
            ix = oi;
        }
    }
}

__global__ void __launch_bounds__(kGibbsThreads) k_gibbs(const GibbsArgs g)
{
    extern __shared__ __align__(16) uint32_t dyn[];
    __shared__ double Wt[kGibbsWaves][20 * 32];
    __shared__ double bgs[20];
    __shared__ int32_t cnt[kGibbsWaves][20 * 32];
    __shared__ int32_t cur[kGibbsWaves][kGibbsMaxT];
    __shared__ int32_t bst[kGibbsWaves][kGibbsMaxT];

    const pm_inst &I = g.one;
    const int tid = threadIdx.x, wv = tid / kWave, lane = lane_id();
    const int A = g.A, l = g.l, AL = A * l, t = I.t;
    uint32_t *seq = dyn;
    int64_t *offs = reinterpret_cast<int64_t *>(dyn + ((g.seq_cap + 1) & ~1));
    const int seq_words = g.seq_cap ? (int)(A == 4 ? (I.n_total + 15) / 16 + 4 : (I.n_total + 5) / 6 + 4) : 0;
    for (int i = tid; i < seq_words; i += kGibbsThreads) seq[i] = I.packed[i];
    if (g.off_cap)
        for (int i = tid; i <= t; i += kGibbsThreads) offs[i] = I.offsets[i];
    for (int c = tid; c < A; c += kGibbsThreads) bgs[c] = g.bg[c];
    __syncthreads();
    const uint32_t *W = g.seq_cap ? seq : I.packed;
    const int64_t *O = g.off_cap ? offs : I.offsets;

    int64_t nvalid = g.n_dev ? *g.n_dev : g.B;
    if (nvalid > g.B) nvalid = g.B;
    const int64_t b = (int64_t)blockIdx.x * kGibbsWaves + wv;
    if (b >= nvalid) return;  // whole waves leave; no workgroup barrier follows

    double *Tw = Wt[wv];
    int32_t *n = cnt[wv];
    int32_t *cs = cur[wv];
    int32_t *bs = bst[wv];
    const double beta = g.beta;

    // start: the best start of every sequence under theta0 (first on ties)
    for (int e = lane; e < AL; e += kWave) Tw[e] = log(g.theta0[b * AL + e]) - log(bgs[e / l]);
    __builtin_amdgcn_wave_barrier();
    for (int i = 0; i < t; ++i) {
        const int64_t s0 = O[i], L = O[i + 1] - s0 - l + 1;
        double bv = -INFINITY;
        int64_t ba = INT64_MAX;
        for (int64_t a = lane; a < L; a += kWave) {
            const double v = start_score(A, W, s0, a, Tw, l);
            if (v > bv) {
                bv = v;
                ba = a;
            }
        }
        wave_argmax(bv, ba);
        if (lane == 0) cs[i] = (int32_t)ba;
    }
    for (int e = lane; e < AL; e += kWave) n[e] = 0;
    __builtin_amdgcn_wave_barrier();
    for (int i = 0; i < t; ++i)
        if (lane < l) atomicAdd(&n[sym_at(A, W, O[i] + cs[i] + lane) * l + lane], 1);
    __builtin_amdgcn_wave_barrier();
    double Fb = alignment_F(n, bgs, A, l, t, beta);
    const int it1 = g.sweeps + 1;
    if (g.F && lane == 0) g.F[b * it1] = Fb;
    for (int i = lane; i < t; i += kWave) bs[i] = cs[i];

    const double tm1 = (double)(t - 1) + beta;
    for (int r = 0; r < g.sweeps; ++r) {
        for (int i = 0; i < t; ++i) {
            const int64_t s0 = O[i], L = O[i + 1] - s0 - l + 1;
            // the other t-1 sites' model
            __builtin_amdgcn_wave_barrier();
            if (lane < l) atomicSub(&n[sym_at(A, W, s0 + cs[i] + lane) * l + lane], 1);
            __builtin_amdgcn_wave_barrier();
            for (int e = lane; e < AL; e += kWave) {
                const int c = e / l;
                Tw[e] = log(((double)n[e] + beta * bgs[c]) / tm1) - log(bgs[c]);
            }
            __builtin_amdgcn_wave_barrier();
            // lane chunks of consecutive starts
            const int64_t C = (L + kWave - 1) / kWave;
            const int64_t a0 = min(L, (int64_t)lane * C), a1 = min(L, a0 + C);
            double mx = -INFINITY;
            for (int64_t a = a0; a < a1; ++a) mx = fmax(mx, start_score(A, W, s0, a, Tw, l));
            mx = wave_max(mx);
            double part = 0;
            for (int64_t a = a0; a < a1; ++a) part += exp(start_score(A, W, s0, a, Tw, l) - mx);
            // running sums over the lanes in start order
            double incl = part;
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                const double v = __shfl_up(incl, o);
                if (lane >= o) incl += v;
            }
            const double tot = __shfl(incl, kWave - 1);
            const double target = gibbs_uniform(g.seed, r, i, b) * tot;
            const uint64_t over = __ballot(incl > target);
            int64_t pick = L - 1;
            if (over) {
                const int who = __builtin_ctzll(over);
                int64_t found = L - 1;
                if (lane == who) {
                    double run = incl - part;
                    for (int64_t a = a0; a < a1; ++a) {
                        run += exp(start_score(A, W, s0, a, Tw, l) - mx);
                        if (run > target) {
                            found = a;
                            break;
                        }
                    }
                }
                pick = __shfl(found, who);
            }
            if (lane == 0) cs[i] = (int32_t)pick;
            __builtin_amdgcn_wave_barrier();
            if (lane < l) atomicAdd(&n[sym_at(A, W, s0 + pick + lane) * l + lane], 1);
            __builtin_amdgcn_wave_barrier();
        }
        const double Fr = alignment_F(n, bgs, A, l, t, beta);
        if (g.F && lane == 0) g.F[b * it1 + r + 1] = Fr;
        if (Fr > Fb) {
            Fb = Fr;
            for (int i = lane; i < t; i += kWave) bs[i] = cs[i];
        }
        __builtin_amdgcn_wave_barrier();
    }
    // the best alignment's model and sites
    for (int e = lane; e < AL; e += kWave) n[e] = 0;
    __builtin_amdgcn_wave_barrier();
    for (int i = 0; i < t; ++i)
        if (lane < l) atomicAdd(&n[sym_at(A, W, O[i] + bs[i] + lane) * l + lane], 1);
    __builtin_amdgcn_wave_barrier();
    for (int e = lane; e < AL; e += kWave)
        g.theta_out[b * AL + e] = ((double)n[e] + beta * bgs[e / l]) / ((double)t + beta);
    if (g.sites)
        for (int i = lane; i < t; i += kWave) g.sites[b * t + i] = bs[i];
}

}  // namespace pm

using namespace pm;

extern "C" int gibbs_refine(const pm_seqs *S, int32_t l, const double *theta0, const double *bg, int64_t B,
                            const int64_t *n_dev, int32_t sweeps, double beta, uint64_t seed, double *theta_out,
                            double *F_out, int32_t *sites_out, void *stream)
{
    clear_error();
    int rc = check_seqs(S, l);
    if (rc) return rc;
    if (B < 0 || sweeps < 0) return fail(PM_EINVAL, "need B >= 0 and sweeps >= 0");
    if (!(beta > 0)) return fail(PM_EINVAL, "Gibbs sampling needs beta > 0 (a start's weight would be 0)");
    if (S->t > kGibbsMaxT) return fail(PM_ERANGE, "t = %d above the sampler's %d sequences", S->t, kGibbsMaxT);
    if (B > ((int64_t)1 << 36)) return fail(PM_ERANGE, "B too large");
    if (B > 0 && (!theta0 || !bg || !theta_out)) return fail(PM_EINVAL, "NULL buffer");
    if (B == 0) return PM_OK;
    GibbsArgs g{};
    g.one = inst_of(S, l);
    g.theta0 = theta0;
    g.bg = bg;
    g.n_dev = n_dev;
    g.theta_out = theta_out;
    g.F = F_out;
    g.sites = sites_out;
    g.B = B;
    g.l = l;
    g.A = S->alphabet;
    g.sweeps = sweeps;
    g.beta = beta;
    g.seed = seed;
    const int64_t nw = pm_packed_words(S->alphabet, S->n_total);
    g.seq_cap = nw * 4 <= 48 * 1024 ? (int)nw : 0;
    g.off_cap = (S->t + 1) * 8 <= 8 * 1024 ? S->t + 1 : 0;
    const size_t lds = ((g.seq_cap + 1) & ~1) * 4 + (size_t)g.off_cap * 8;
    const int64_t blocks = (B + kGibbsWaves - 1) / kGibbsWaves;
    hipLaunchKernelGGL(k_gibbs, dim3((unsigned)blocks), dim3(kGibbsThreads), lds, as_stream(stream), g);
    PM_LAUNCHED();
    return PM_OK;
}
