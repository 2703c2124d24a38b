// a7 - a9 for protein models on the matrix cores: the precision form with a
// 20-letter one-hot.
//
// E-step scores of a tile of 16 windows for 16 models: S = OneHot . W with
// contraction index kappa = 20 p + sigma (position p, letter sigma), 20 l of
// them padded to KS steps of 32.  M-step counts: C = OneHot^T . Z with the
// contraction over 32 windows (two E tiles), 2 KS row tiles of 16 kappa rows.
// v_mfma_f32_16x16x32_f16, one FP16 value per non-0/1 operand (the log-odds W
// and the posteriors Z), FP32 accumulation.  The per-sequence log-sum-exp is
// FP64: each lane keeps an FP64 sum of its terms 2^(S - ref) against a
// whole-number reference (so that moving it rescales the sum exactly), the
// lanes of a model are combined in FP64 and the logarithm is FP64; LLR and J
// are FP64.
//
// A 20-letter model has 20 l count rows, too many to keep one sequence's
// unnormalised counts beside the running totals, so every iteration first
// sweeps the sequences for their log-sum-exp (kept in LDS; in the final E-step
// also the best start), then sweeps them again with exactly normalised
// posteriors feeding M-step accumulators that stay in registers across the
// sequences.  Beyond 8 contraction steps the count rows are split over two
// such sweeps, which keeps the accumulators and the log-odds in registers
// (no spills) at the cost of one more E-step per window pair.
//
// Lane layout (lane L, r = L % 16, g = L / 16), as for the DNA kernel:
//   E-step A: window row r, kappa 32 ks + 8 g .. + 7;  B: model r, same kappa;
//   D: model r, windows 4g .. 4g+3 of the tile;
//   M-step A: kappa row 16 rt + r, windows w_j (j < 8) = 4g + j (tile 0) and
//   16 + 4g + j - 4 (tile 1), exactly the windows of the lane's E-step
//   outputs, which therefore feed the M-step B operand without moving.
// A workgroup of four waves takes 64 models of one instance; the tables of a
// window pair are built by the whole workgroup in LDS from the sequence's
// symbols unpacked to bytes.
#include <math.h>

#include "pm_common.h"

namespace pm {

typedef _Float16 half8p __attribute__((ext_vector_type(8)));
typedef float float4p __attribute__((ext_vector_type(4)));

constexpr int kPW = 4;           // waves per workgroup
constexpr int kPSymMax = 2048;   // longest sequence (symbols)
constexpr int kPTMax = 64;       // most sequences
constexpr float kPLog2e = 1.4426950408889634f;
constexpr int kPOneSweepKS = 14;  // largest KS whose 2 KS count tiles and LDS tables fit two workgroups

struct EmProtArgs {
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
    int t, l, iters;
    double beta;
};

template <int KS, int RH>
struct ProtTables {
    uint4 e[2][KS][64];  // E-step A fragments of the two tiles
    uint4 m[RH][64];     // M-step A fragments of the sweep's row tiles
};

// eight FP16 halves, 1.0 at the set bits of an 8-bit mask
__device__ __forceinline__ uint4 mask8_halves(uint32_t mk)
{
    uint32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
        w[q] = (((mk >> (2 * q)) & 1u) ? 0x3C00u : 0u) | (((mk >> (2 * q + 1)) & 1u) ? 0x3C000000u : 0u);
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// tables of the window pair starting at a0 (sequence-relative), sym = the
// sequence's symbols as bytes; with h >= 0 also the M-step fragments of the
// row tiles h RH .. h RH + RH - 1
template <int KS, int RH>
__device__ __forceinline__ void build_prot_tables(const uint8_t *sym, int a0, int l, int h, ProtTables<KS, RH> &T,
                                                  uint32_t *mm)
{
    const int nk = 20 * l;
    for (int e = threadIdx.x; e < 2 * KS * 64; e += 64 * kPW) {
        const int lane = e & 63, ks = (e >> 6) % KS, tile = (e >> 6) / KS;
        const int r = lane & 15, g = lane >> 4;
        const int w = a0 + 16 * tile + r;
        const int k0 = 32 * ks + 8 * g;
        uint32_t mk = 0;
        if (k0 < nk) {
            const int p0 = k0 / 20, p1 = (k0 + 7) / 20;
            const int i0 = 20 * p0 + sym[w + p0] - k0;
            if (i0 >= 0 && i0 < 8) mk |= 1u << i0;
            if (p1 != p0 && p1 < l) {
                const int i1 = 20 * p1 + sym[w + p1] - k0;
                if (i1 >= 0 && i1 < 8) mk |= 1u << i1;
            }
            // kappa >= 20 l never matches: p1 < l guards the second position
        }
        T.e[tile][ks][lane] = mask8_halves(mk);
    }
    if (h < 0) return;
    // M-step fragments by scattering each (window, position) symbol to its
    // kappa row: word mm[kappa - 16 RH h] holds, in byte g, the windows of
    // lane group g
    const int kb = 16 * RH * h;
    for (int q = threadIdx.x; q < 16 * RH; q += 64 * kPW) mm[q] = 0;
    __syncthreads();
    for (int q = threadIdx.x; q < 32 * l; q += 64 * kPW) {
        const int p = q >> 5, jj = q & 31, g = jj >> 3, j = jj & 7;
        const int w = a0 + (j < 4 ? 4 * g + j : 16 + 4 * g + j - 4);
        const int kr = 20 * p + sym[w + p] - kb;
        if (kr >= 0 && kr < 16 * RH) atomicOr(mm + kr, 1u << (8 * g + j));
    }
    __syncthreads();
    for (int e = threadIdx.x; e < RH * 64; e += 64 * kPW) {
        const int lane = e & 63, rt = e >> 6;
        const int r = lane & 15, g = lane >> 4;
        const int kap = kb + 16 * rt + r;
        T.m[rt][lane] = mask8_halves(kap < nk ? (mm[16 * rt + r] >> (8 * g)) & 0xffu : 0u);
    }
}

// NH sweeps of the M-step per iteration, each over RH = 2 KS / NH row tiles
template <int KS, int NH>
__global__ void __launch_bounds__(64 * kPW, 2) k_em_prot(const EmProtArgs a)
{
    constexpr int RH = (2 * KS + NH - 1) / NH;
    // the tables share LDS with the staging of the log-odds (each lane reads
    // back only what it wrote, before the first table build of the iteration)
    __shared__ __align__(16) union {
        ProtTables<KS, RH> T;
        uint4 w[kPW][KS][64];
    } U;
    ProtTables<KS, RH> &T = U.T;
    __shared__ uint8_t sym[kPSymMax + 64];
    __shared__ uint32_t mm[16 * RH];    // M-step table build: window masks per kappa row
    __shared__ float lzs[kPW][16][kPTMax];  // per-sequence log2-sum-exp2 of every model
    __shared__ double lbg[20];              // ln of the background frequencies

    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
    int64_t nvalid = a.n_dev ? *a.n_dev : a.B;
    if (nvalid > a.B) nvalid = a.B;
    const int64_t b0 = (int64_t)blockIdx.x * 16 * kPW;
    if (b0 >= nvalid) return;  // uniform over the workgroup
    const int l = a.l, t = a.t, AL = 20 * l, nk = 20 * l;
    const int64_t b = b0 + 16 * wv + r;
    const bool vb = b < nvalid;
    const double beta = a.beta;
    if (threadIdx.x < 20) lbg[threadIdx.x] = log(a.bg[threadIdx.x]);
    __syncthreads();

    auto unpack = [&](int i, int &L) {
        const int64_t s0 = a.offsets[i];
        const int n = (int)(a.offsets[i + 1] - s0);
        L = n - l + 1;
        __syncthreads();  // the previous users of sym and T are done
        for (int q = threadIdx.x; q < n + 64; q += 64 * kPW)
            sym[q] = q < n ? (uint8_t)prot_sym(a.packed, s0 + q) : (uint8_t)0;
    };
    auto estep = [&](const half8p(&Wb)[KS], float4p &S0, float4p &S1) {
        S0 = float4p{0.f, 0.f, 0.f, 0.f};
        S1 = S0;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const half8p A0 = __builtin_bit_cast(half8p, T.e[0][ks][lane]);
            const half8p A1 = __builtin_bit_cast(half8p, T.e[1][ks][lane]);
            S0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(A0, Wb[ks], S0, 0, 0, 0);
            S1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(A1, Wb[ks], S1, 0, 0, 0);
        }
    };

    half8p Wb[KS];
    for (int it = 0; it <= a.iters; ++it) {
        const bool last = it == a.iters;
        const double *src = it == 0 ? a.theta0 : a.theta_out;
        // ---- log-odds of the lane's B-operand entries (log2 units) and the
        // prior, one contraction step at a time through LDS (an unrolled build
        // would keep the loads of all 8 KS entries in flight in registers)
        double prior = 0;
#pragma unroll 1
        for (int ks = 0; ks < KS; ++ks) {
            half8p hv;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int kap = 32 * ks + 8 * g + j;
                float w = 0.f;
                if (kap < nk && vb) {
                    const int p = kap / 20, sg = kap - 20 * p;
                    const double th = src[b * AL + sg * l + p];
                    if (it == 0) a.theta_out[b * AL + sg * l + p] = th;
                    const double lt = log(th);
                    w = (float)((lt - lbg[sg]) * (double)kPLog2e);
                    prior += a.bg[sg] * lt;
                }
                hv[j] = (_Float16)w;
            }
            U.w[wv][ks][lane] = __builtin_bit_cast(uint4, hv);
        }
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) Wb[ks] = __builtin_bit_cast(half8p, U.w[wv][ks][lane]);
        prior += __shfl_xor(prior, 16);
        prior += __shfl_xor(prior, 32);

        // ---- first sweep: log-sum-exp of every sequence (the best start too in
        // the final E-step)
        double llr = 0;
        for (int i = 0; i < t; ++i) {
            int L;
            unpack(i, L);
            // mx: a whole number at or above every score seen by this lane
            // (-inf before the first); sm: FP64 sum of 2^(v - mx)
            float mx = -INFINITY, bestv = -INFINITY;
            double sm = 0.0;
            int besti = 0;
            for (int a0 = 0; a0 < L; a0 += 32) {
                __syncthreads();
                build_prot_tables<KS, RH>(sym, a0, l, -1, T, mm);
                __syncthreads();
                float4p S0, S1;
                estep(Wb, S0, S1);
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int w = a0 + 16 * (q >> 2) + 4 * g + (q & 3);
                    const float v = q < 4 ? S0[q & 3] : S1[q & 3];
                    if (w < L) {
                        if (v > mx) {
                            const float nm = ceilf(v);
                            sm = mx > -INFINITY ? ldexp(sm, (int)(mx - nm)) : 0.0;
                            mx = nm;
                        }
                        sm += (double)__builtin_amdgcn_exp2f(v - mx);
                        if (last && v > bestv) {
                            bestv = v;
                            besti = w;
                        }
                    }
                }
            }
            // combine the four lanes of each model in FP64 (the references are
            // whole numbers: the rescales are exact)
            float M = mx;
            M = fmaxf(M, __shfl_xor(M, 16));
            M = fmaxf(M, __shfl_xor(M, 32));
            double part = mx > -INFINITY ? ldexp(sm, (int)(mx - M)) : 0.0;
            part += __shfl_xor(part, 16);
            part += __shfl_xor(part, 32);
            const double lz = (double)M + log2(part);  // log2 of the sum of 2^S
            if (g == 0) lzs[wv][r][i] = (float)lz;
            llr += lz * 0.6931471805599453 - log((double)L);
            if (last && a.sites) {
#pragma unroll
                for (int o = 16; o <= 32; o <<= 1) {
                    const float ov = __shfl_xor(bestv, o);
                    const int oi = __shfl_xor(besti, o);
                    if (ov > bestv || (ov == bestv && oi < besti)) {
                        bestv = ov;
                        besti = oi;
                    }
                }
                if (g == 0 && vb) a.sites[b * t + i] = besti;
            }
        }
        if (g == 0 && vb) {
            a.J[b * (a.iters + 1) + it] = llr + beta * prior;
            if (a.llr) a.llr[b * (a.iters + 1) + it] = llr;
        }
        if (last) break;

        // ---- NH more sweeps: exactly normalised posteriors into the M-step
        // counts of RH row tiles each, kept in registers across the sequences
        __syncthreads();  // every lane has read its theta^it entries; lzs visible
        for (int h = 0; h < NH; ++h) {
            float4p C[RH];
#pragma unroll
            for (int rt = 0; rt < RH; ++rt) C[rt] = float4p{0.f, 0.f, 0.f, 0.f};
            for (int i = 0; i < t; ++i) {
                int L;
                unpack(i, L);
                const float lz = lzs[wv][r][i];
                for (int a0 = 0; a0 < L; a0 += 32) {
                    __syncthreads();
                    build_prot_tables<KS, RH>(sym, a0, l, h, T, mm);
                    __syncthreads();
                    float4p S0, S1;
                    estep(Wb, S0, S1);
                    half8p Ph;
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        const int w = a0 + 16 * (q >> 2) + 4 * g + (q & 3);
                        const float v = q < 4 ? S0[q & 3] : S1[q & 3];
                        Ph[q] = (_Float16)(w < L ? __builtin_amdgcn_exp2f(v - lz) : 0.f);
                    }
#pragma unroll
                    for (int rt = 0; rt < RH; ++rt) {
                        const half8p Am = __builtin_bit_cast(half8p, T.m[rt][lane]);
                        C[rt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Am, Ph, C[rt], 0, 0, 0);
                    }
                }
            }
            // counts of the lane's rows, kappa = 16 (h RH + rt) + 4 g + q; the
            // base goes through an empty asm statement so that the addresses of
            // these stores are formed here, not hoisted to the kernel's entry
            // and held (spilled) across the sweeps
            int g4 = 16 * h * RH + 4 * g;
            asm volatile("" : "+v"(g4));
            if (vb) {
#pragma unroll
                for (int rt = 0; rt < RH; ++rt)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int kap = g4 + 16 * rt + q;
                        if (kap < nk) {
                            const int p = kap / 20, sg = kap - 20 * p;
                            a.theta_out[b * AL + sg * l + p] = (double)C[rt][q];
                        }
                    }
            }
        }
        // ---- every column of the model divided by its own total; lane g takes
        // the columns p = g, g + 4, ...
        __syncthreads();
        if (vb)
            for (int p = g; p < l; p += 4) {
                double s = 0;
                for (int c = 0; c < 20; ++c) s += a.theta_out[b * AL + c * l + p];
                const double tot = s + beta;
                for (int c = 0; c < 20; ++c)
                    a.theta_out[b * AL + c * l + p] = (a.theta_out[b * AL + c * l + p] + beta * a.bg[c]) / tot;
            }
        __syncthreads();  // theta^(it+1) visible to every lane before it is read
    }
}

template <int KS>
static int launch_prot(const EmProtArgs &a, hipStream_t st)
{
    // one M-step sweep while the counts of all 2 KS row tiles fit in registers
    // beside the log-odds, two beyond
    constexpr int NH = KS <= kPOneSweepKS ? 1 : 2;
    const int64_t groups = (a.B + 16 * kPW - 1) / (16 * kPW);
    hipLaunchKernelGGL((k_em_prot<KS, NH>), dim3((unsigned)groups), dim3(64 * kPW), 0, st, a);
    PM_LAUNCHED();
    return PM_OK;
}

int em_refine_prot(const pm_seqs *S, int32_t l, const double *theta0, const double *bg, int64_t B,
                   const int64_t *n_dev, int32_t iters, double beta, double *theta_out, double *J_out,
                   double *llr_out, int32_t *sites_out, hipStream_t st)
{
    if (l > 24) return fail(PM_ERANGE, "the protein matrix-core form takes l <= 24");
    if (S->t > kPTMax) return fail(PM_ERANGE, "the protein matrix-core form takes t <= %d", kPTMax);
    if (S->n_max > kPSymMax) return fail(PM_ERANGE, "the protein matrix-core form takes n_i <= %d", kPSymMax);
    EmProtArgs a{};
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
    a.t = S->t;
    a.l = l;
    a.iters = iters;
    a.beta = beta;
    switch ((20 * l + 31) / 32) {
    case 1: return launch_prot<1>(a, st);
    case 2: return launch_prot<2>(a, st);
    case 3: return launch_prot<3>(a, st);
    case 4: return launch_prot<4>(a, st);
    case 5: return launch_prot<5>(a, st);
    case 6: return launch_prot<6>(a, st);
    case 7: return launch_prot<7>(a, st);
    case 8: return launch_prot<8>(a, st);
    case 9: return launch_prot<9>(a, st);
    case 10: return launch_prot<10>(a, st);
    case 11: return launch_prot<11>(a, st);
    case 12: return launch_prot<12>(a, st);
    case 13: return launch_prot<13>(a, st);
    case 14: return launch_prot<14>(a, st);
    default: return launch_prot<15>(a, st);
    }
}

}  // namespace pm
