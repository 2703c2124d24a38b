// a7 - a9 on the matrix cores: OOPS EM of DNA models as one-hot contractions.
//
// For a tile of windows and a group of 16 models the E-step scores are a
// product of the windows' one-hot encoding (4l columns, entries 0/1) with the
// models' log-odds (4l x 16):  S = OneHot . W.  The M-step counts are the
// transposed product with the posteriors:  C = OneHot^T . P.  Per sequence
// the posteriors are a softmax over windows, so one pass over a sequence is
// an attention-like sweep with a running maximum and rescaled accumulators.
//
// Arithmetic: v_mfma_f32_16x16x32_f16.  The one-hot side is exact in FP16.
// The other side is split in two FP16 halves, x = hi + lo with
// hi = fp16(x) and lo = fp16(x - hi), and both halves accumulate into the
// same FP32 accumulator, so every product is exact and the operand carries
// about 22 significant bits; sums are FP32.  Scores are kept in log2 units
// (W scaled by log2 e) so the softmax uses the hardware exp2; the per-sequence
// log-sum-exp and the objective are formed in FP64.
//
// Lane layout of one 16x16x32 MFMA (lane L, r = L % 16, g = L / 16):
//   A operand: row r, the g-th group of 8 contraction indices;
//   B operand: column r, the same 8 contraction indices;
//   D:         column r, rows 4g .. 4g+3.
// E-step: rows = 16 windows, columns = 16 models, contraction = (position,
// letter) pairs, position-major.  Lane (r, g) of k-block kb carries positions
// 8kb+2g and 8kb+2g+1.  M-step: rows = 16 (position, letter) pairs, columns =
// models, contraction = 32 windows (two E tiles); lane (r, g) carries windows
// 4g..4g+3 of the first tile and of the second, exactly the rows its E-step
// outputs hold, so posteriors feed the M-step without leaving registers.
#include <math.h>

#include "pm_common.h"

namespace pm {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float float4v __attribute__((ext_vector_type(4)));

struct EmMfmaArgs {
    const uint32_t *packed;
    const int64_t *offsets;
    const double *theta0;
    const double *bg;
    const int64_t *n_dev;
    double *theta_out;
    double *J;
    double *llr;
    int32_t *sites;
    int64_t B;
    int64_t nwords;  // packed words (reads are clamped below this)
    int t, l, iters;
    double beta;
};

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kPScale = 11.0f;  // posteriors are scaled by 2^11 before the split

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t ld_clamped(const uint32_t *w, int64_t i, int64_t nw)
{
    return w[i < nw ? i : nw - 1];
}

// 16 DNA symbols starting at P (MSB-first), reads clamped to the buffer
__device__ __forceinline__ uint32_t dna16(const uint32_t *w, int64_t P, int64_t nw)
{
    const int64_t wi = P >> 4;
    const uint32_t r = (uint32_t)(P & 15) << 1;
    const uint64_t v = ((uint64_t)ld_clamped(w, wi, nw) << 32) | ld_clamped(w, wi + 1, nw);
    return (uint32_t)(v >> (32 - r));
}

// two FP16 halves (1.0 where letter == c) for letter codes a (low half) and b
__device__ __forceinline__ uint32_t onehot_pair(uint32_t a, uint32_t b, uint32_t c)
{
    return (a == c ? 0x3C00u : 0u) | (b == c ? 0x3C000000u : 0u);
}

__device__ __forceinline__ uint32_t pack_h2(_Float16 x, _Float16 y)
{
    return (uint32_t)__builtin_bit_cast(uint16_t, x) | ((uint32_t)__builtin_bit_cast(uint16_t, y) << 16);
}

template <int LB, int NG>
__global__ void __launch_bounds__(64) k_em_mfma(const EmMfmaArgs a)
{
    constexpr int MTX = 2 * LB;  // M-tiles of 4 positions each, at most
    constexpr int PX = 8 * LB;   // positions covered by the E-step k-blocks
    __shared__ __align__(16) uint32_t oh2[64][4];     // one-hot of symbols e, e+1
    __shared__ __align__(16) uint32_t mt4[64][4][2];  // [e][c]: symbols e..e+3 == c
    __shared__ __align__(16) float acc[NG][16][PX][4];

    const int lane = threadIdx.x, r = lane & 15, g = lane >> 4;
    int64_t nvalid = a.n_dev ? *a.n_dev : a.B;
    if (nvalid > a.B) nvalid = a.B;
    const int64_t b0 = (int64_t)blockIdx.x * 16 * NG;
    if (b0 >= nvalid) return;
    const int l = a.l, t = a.t, AL = 4 * l;
    const int MT = (l + 3) >> 2;
    const double beta = a.beta;
    const double lbg[4] = {log(a.bg[0]), log(a.bg[1]), log(a.bg[2]), log(a.bg[3])};

    half8 Whi[NG][LB], Wlo[NG][LB];
    float4v O[NG][MTX];

    for (int it = 0; it <= a.iters; ++it) {
        const bool last = it == a.iters;
        const double *src = it == 0 ? a.theta0 : a.theta_out;
        double prior[NG], llr[NG];
        // ---- log-odds of every model (own entries: positions p = 4mt + g)
#pragma unroll
        for (int grp = 0; grp < NG; ++grp) {
            const int64_t b = b0 + 16 * grp + r;
            const bool vb = b < nvalid;
            double pr = 0;
#pragma unroll
            for (int mt = 0; mt < MTX; ++mt) {
                const int p = 4 * mt + g;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    float w = 0.f;
                    if (p < l && vb) {
                        const double th = src[b * AL + c * l + p];
                        if (it == 0) a.theta_out[b * AL + c * l + p] = th;
                        w = (float)((log(th) - lbg[c]) * (double)kLog2e);
                        pr += a.bg[c] * log(th);
                    }
                    if (p < PX) acc[grp][r][p][c] = w;
                }
            }
            pr += __shfl_xor(pr, 16);
            pr += __shfl_xor(pr, 32);
            prior[grp] = pr;
            llr[grp] = 0;
        }
        wave_sync();
        // ---- B operands of the E-step: positions 8kb+2g, 8kb+2g+1, letters 0..3
#pragma unroll
        for (int grp = 0; grp < NG; ++grp)
#pragma unroll
            for (int kb = 0; kb < LB; ++kb) {
                const int p0 = 8 * kb + 2 * g;
                const float4v u = *reinterpret_cast<const float4v *>(&acc[grp][r][p0][0]);
                const float4v v = *reinterpret_cast<const float4v *>(&acc[grp][r][p0 + 1][0]);
                half8 hi, lo;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    hi[q] = (_Float16)u[q];
                    lo[q] = (_Float16)(u[q] - (float)hi[q]);
                    hi[q + 4] = (_Float16)v[q];
                    lo[q + 4] = (_Float16)(v[q] - (float)hi[q + 4]);
                }
                Whi[grp][kb] = hi;
                Wlo[grp][kb] = lo;
            }
        wave_sync();
        // ---- clear the count accumulators (own entries)
#pragma unroll
        for (int grp = 0; grp < NG; ++grp)
#pragma unroll
            for (int mt = 0; mt < MTX; ++mt) {
                const int p = 4 * mt + g;
                if (p < PX) *reinterpret_cast<float4v *>(&acc[grp][r][p][0]) = float4v{0.f, 0.f, 0.f, 0.f};
            }

        for (int i = 0; i < t; ++i) {
            const int64_t s0 = a.offsets[i];
            const int L = (int)(a.offsets[i + 1] - s0) - l + 1;
            float mrun[NG], srun[NG], bestv[NG];
            int besti[NG];
#pragma unroll
            for (int grp = 0; grp < NG; ++grp) {
                mrun[grp] = -INFINITY;
                srun[grp] = 0.f;
                bestv[grp] = -INFINITY;
                besti[grp] = 0;
#pragma unroll
                for (int mt = 0; mt < MTX; ++mt) O[grp][mt] = float4v{0.f, 0.f, 0.f, 0.f};
            }
            for (int a0 = 0; a0 < L; a0 += 32) {
                // ---- tables for the symbols at s0 + a0 + e, e = 0..63 (+3)
                {
                    const uint32_t w16 = dna16(a.packed, s0 + a0 + lane, a.nwords);
                    const uint32_t s_0 = w16 >> 30, s_1 = (w16 >> 28) & 3u, s_2 = (w16 >> 26) & 3u,
                                   s_3 = (w16 >> 24) & 3u;
                    uint32_t e0 = onehot_pair(s_0, s_0, 0) & 0xffffu;
                    e0 |= onehot_pair(s_0, s_0, 1) & 0xffff0000u;
                    uint32_t e1 = onehot_pair(s_0, s_0, 2) & 0xffffu;
                    e1 |= onehot_pair(s_0, s_0, 3) & 0xffff0000u;
                    uint32_t e2 = onehot_pair(s_1, s_1, 0) & 0xffffu;
                    e2 |= onehot_pair(s_1, s_1, 1) & 0xffff0000u;
                    uint32_t e3 = onehot_pair(s_1, s_1, 2) & 0xffffu;
                    e3 |= onehot_pair(s_1, s_1, 3) & 0xffff0000u;
                    *reinterpret_cast<uint4 *>(&oh2[lane][0]) = make_uint4(e0, e1, e2, e3);
#pragma unroll
                    for (uint32_t c = 0; c < 4; ++c)
                        *reinterpret_cast<uint2 *>(&mt4[lane][c][0]) =
                            make_uint2(onehot_pair(s_0, s_1, c), onehot_pair(s_2, s_3, c));
                }
                wave_sync();
                half8 Ae[2][LB], Am[MTX];
#pragma unroll
                for (int T = 0; T < 2; ++T)
#pragma unroll
                    for (int kb = 0; kb < LB; ++kb)
                        Ae[T][kb] = *reinterpret_cast<const half8 *>(&oh2[16 * T + r + 8 * kb + 2 * g][0]);
                if (!last) {
                    // M-step A operand: row (position pm, letter cm), windows 4g..4g+3
                    // of both tiles
#pragma unroll
                    for (int mt = 0; mt < MTX; ++mt) {
                        const int pm = 4 * mt + (r >> 2), cm = r & 3;
                        uint4 uu = make_uint4(0, 0, 0, 0);
                        if (mt < MT) {
                            const uint2 u0 = *reinterpret_cast<const uint2 *>(&mt4[4 * g + pm][cm][0]);
                            const uint2 u1 = *reinterpret_cast<const uint2 *>(&mt4[16 + 4 * g + pm][cm][0]);
                            uu = make_uint4(u0.x, u0.y, u1.x, u1.y);
                        }
                        Am[mt] = __builtin_bit_cast(half8, uu);
                    }
                }
                const bool tail = a0 + 32 > L;
#pragma unroll
                for (int grp = 0; grp < NG; ++grp) {
                    float4v S[2];
#pragma unroll
                    for (int T = 0; T < 2; ++T) {
                        S[T] = float4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                        for (int kb = 0; kb < LB; ++kb) {
                            S[T] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Ae[T][kb], Whi[grp][kb], S[T], 0, 0, 0);
                            S[T] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Ae[T][kb], Wlo[grp][kb], S[T], 0, 0, 0);
                        }
                    }
                    if (tail) {
#pragma unroll
                        for (int T = 0; T < 2; ++T)
#pragma unroll
                            for (int j = 0; j < 4; ++j)
                                if (a0 + 16 * T + 4 * g + j >= L) S[T][j] = -INFINITY;
                    }
                    if (last) {
#pragma unroll
                        for (int T = 0; T < 2; ++T)
#pragma unroll
                            for (int j = 0; j < 4; ++j)
                                if (S[T][j] > bestv[grp]) {
                                    bestv[grp] = S[T][j];
                                    besti[grp] = a0 + 16 * T + 4 * g + j;
                                }
                    }
                    // running maximum over the model's windows
                    float tm = fmaxf(fmaxf(fmaxf(S[0][0], S[0][1]), fmaxf(S[0][2], S[0][3])),
                                     fmaxf(fmaxf(S[1][0], S[1][1]), fmaxf(S[1][2], S[1][3])));
                    tm = fmaxf(tm, __shfl_xor(tm, 16));
                    tm = fmaxf(tm, __shfl_xor(tm, 32));
                    const float mn = fmaxf(mrun[grp], tm);
                    if (__ballot(mn > mrun[grp])) {
                        const float al = __builtin_amdgcn_exp2f(mrun[grp] - mn);
                        srun[grp] *= al;
                        if (!last)
#pragma unroll
                            for (int mt = 0; mt < MTX; ++mt) O[grp][mt] *= al;
                    }
                    mrun[grp] = mn;
                    const float sh = mn - kPScale;
                    float P[8];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        P[j] = __builtin_amdgcn_exp2f(S[0][j] - sh);
                        P[4 + j] = __builtin_amdgcn_exp2f(S[1][j] - sh);
                    }
                    float ps = 0.f;
#pragma unroll
                    for (int q = 0; q < 8; ++q) ps += P[q];
                    srun[grp] += ps;
                    if (!last) {
                        half8 Ph, Pl;
#pragma unroll
                        for (int q = 0; q < 8; ++q) {
                            Ph[q] = (_Float16)P[q];
                            Pl[q] = (_Float16)(P[q] - (float)Ph[q]);
                        }
#pragma unroll
                        for (int mt = 0; mt < MTX; ++mt) {
                            if (mt < MT) {
                                O[grp][mt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Am[mt], Ph, O[grp][mt], 0, 0, 0);
                                O[grp][mt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Am[mt], Pl, O[grp][mt], 0, 0, 0);
                            }
                        }
                    }
                }
                wave_sync();  // the next tile rebuilds the tables
            }
            // ---- end of sequence i: log-sum-exp, counts, sites
#pragma unroll
            for (int grp = 0; grp < NG; ++grp) {
                float sr = srun[grp];
                sr += __shfl_xor(sr, 16);
                sr += __shfl_xor(sr, 32);
                const double lse = (double)mrun[grp] * 0.6931471805599453 + log((double)sr) -
                                   (double)kPScale * 0.6931471805599453;
                llr[grp] += lse - log((double)L);
                if (!last) {
                    const float inv = 1.0f / sr;
#pragma unroll
                    for (int mt = 0; mt < MTX; ++mt) {
                        const int p = 4 * mt + g;
                        if (mt < MT && p < PX) {
                            float4v *dst = reinterpret_cast<float4v *>(&acc[grp][r][p][0]);
                            *dst += O[grp][mt] * inv;
                        }
                    }
                } else if (a.sites) {
                    float bv = bestv[grp];
                    int bi = besti[grp];
#pragma unroll
                    for (int o = 16; o <= 32; o <<= 1) {
                        const float ov = __shfl_xor(bv, o);
                        const int oi = __shfl_xor(bi, o);
                        if (ov > bv || (ov == bv && oi < bi)) {
                            bv = ov;
                            bi = oi;
                        }
                    }
                    const int64_t b = b0 + 16 * grp + r;
                    if (g == 0 && b < nvalid) a.sites[b * t + i] = bi;
                }
            }
        }
        // ---- objective of theta^it, then the M-step (own entries)
#pragma unroll
        for (int grp = 0; grp < NG; ++grp) {
            const int64_t b = b0 + 16 * grp + r;
            if (g == 0 && b < nvalid) {
                a.J[b * (a.iters + 1) + it] = llr[grp] + beta * prior[grp];
                if (a.llr) a.llr[b * (a.iters + 1) + it] = llr[grp];
            }
            if (!last && b < nvalid) {
#pragma unroll
                for (int mt = 0; mt < MTX; ++mt) {
                    const int p = 4 * mt + g;
                    if (p < l) {
                        const float4v cn = *reinterpret_cast<const float4v *>(&acc[grp][r][p][0]);
                        // every column's counts sum to t: normalising by the column's
                        // own total is the same update and stays on the simplex
                        const double tot = (double)cn[0] + (double)cn[1] + (double)cn[2] + (double)cn[3] + beta;
#pragma unroll
                        for (int c = 0; c < 4; ++c)
                            a.theta_out[b * AL + c * l + p] = ((double)cn[c] + beta * a.bg[c]) / tot;
                    }
                }
            }
        }
        wave_sync();
    }
}

template <int LB, int NG>
static int launch_em_mfma(const EmMfmaArgs &a, hipStream_t st)
{
    const int64_t groups = (a.B + 16 * NG - 1) / (16 * NG);
    hipLaunchKernelGGL((k_em_mfma<LB, NG>), dim3((unsigned)groups), dim3(64), 0, st, a);
    PM_LAUNCHED();
    return PM_OK;
}

int em_refine_mfma(const pm_seqs *S, int32_t l, const double *theta0, const double *bg, int64_t B,
                   const int64_t *n_dev, int32_t iters, double beta, double *theta_out, double *J_out,
                   double *llr_out, int32_t *sites_out, hipStream_t st)
{
    EmMfmaArgs a{};
    a.packed = S->packed;
    a.offsets = S->offsets;
    a.theta0 = theta0;
    a.bg = bg;
    a.n_dev = n_dev;
    a.theta_out = theta_out;
    a.J = J_out;
    a.llr = llr_out;
    a.sites = sites_out;
    a.B = B;
    a.nwords = pm_packed_words(S->alphabet, S->n_total);
    a.t = S->t;
    a.l = l;
    a.iters = iters;
    a.beta = beta;
    constexpr int NG = 2;
    switch ((l + 7) / 8) {
    case 1: return launch_em_mfma<1, NG>(a, st);
    case 2: return launch_em_mfma<2, NG>(a, st);
    case 3: return launch_em_mfma<3, NG>(a, st);
    default: return launch_em_mfma<4, NG>(a, st);
    }
}

}  // namespace pm
