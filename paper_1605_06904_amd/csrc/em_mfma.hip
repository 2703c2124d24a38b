// a7 - a9 on the matrix cores: OOPS EM of DNA models as one-hot contractions.
//
// For a tile of windows and a group of 16 models the E-step scores are a
// product of the windows' one-hot encoding (4l columns, entries 0/1) with the
// models' log-odds (4l x 16):  S = OneHot . W.  The M-step counts are the
// transposed product with the posteriors:  C = OneHot^T . P.  Per sequence
// the posteriors are a softmax over windows, so one pass over a sequence is
// an attention-like sweep with a reference maximum and rescaled accumulators.
//
// Arithmetic: v_mfma_f32_16x16x32_f16.  The one-hot side is exact in FP16.
// The other side is split in two FP16 halves, x = hi + lo with
// hi = fp16(x) and lo = fp16(x - hi), both multiplied by the same one-hot
// operand, so every product is exact and the operand carries about 22
// significant bits; sums are FP32.  The single-FP16 form (SPLIT = false) keeps
// only hi: half the matrix-core work, 11-bit operands.  Scores are kept in
// log2 units (W = log2 theta - log2 bg by the hardware FP32 logarithm, about
// 2^-23 relative, inside the 22 bits the split halves carry; the prior term of
// J adds those logarithms in FP64) so the softmax uses the hardware exp2.  The per-sequence
// log-sum-exp is FP64: the posterior terms 2^(S - ref) are FP32 exp2 of FP32
// scores; the eight a lane holds for one window pair are added in FP32 (three
// levels), and these pair partials are accumulated over the whole sequence in
// FP64, so the error does not grow with the sequence length; the four lane
// groups are combined with FP64 shuffles and the logarithm is FP64, as are
// the objective and the final comparison.
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
//
// Softmax reference: scores leave the E-step already shifted by the current
// reference (the accumulator starts at -reference), and the reference moves
// only when a score passes it by more than kSlack, so the common path needs
// neither a cross-lane maximum nor a rescale.  Posteriors enter the M-step as
// 2^(S - ref + kPOff) <= 2^(kPOff + kSlack) = 2^15, inside the FP16 range.
// The reference moves by whole numbers, so every rescale (of the count
// accumulators and of the FP64 sums) is an exact power of two.
//
// Work split: a workgroup of four waves takes 64 G models of one instance, G
// groups of 16 per wave; the groups of a wave share every A operand (the
// one-hot tables), so G = 2 halves the table reads and builds per model and
// gives each wave two independent E-step/softmax/M-step chains to interleave.
// The four waves sweep the same windows in step; the one-hot tables of PPB
// window pairs sit in LDS per step (double-buffered, one barrier per PPB
// pairs).  With a workspace, k_em_tables builds every pair's tables once per
// call and the EM kernel copies each step's into LDS, loading the next step's
// while it computes; without one, the workgroup builds them itself from the
// packed instance in global memory.  (G, PPB) is the tunable tile
// shape: em_autotune times the variants on the caller's models and records
// the fastest per (ceil(l/4), precision) class.
#include <math.h>
#include <stddef.h>
#include <stdlib.h>

#include "pm_common.h"

namespace pm {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef float float4v __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));  // one 16-byte table quad

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
    int site_stride; // sites row length (t, or the largest t of a batch)
    int split;       // 1: two FP16 halves per operand; 0: one FP16 value
    double beta;
    // batch: the instance table and the workgroup plan (k_em_plan), or NULL
    const pm_inst *inst;
    const int64_t *plan;
    int P;
    // precomputed one-hot tables (k_em_tables), or NULL to build them in the
    // kernel; tbase: first slot of every instance of a batch (NULL: one instance)
    const uint8_t *tables;
    const int64_t *tbase;
};

// workgroups of a launch that takes mw models per workgroup: whole groups of
// the B models, or, for a batch, the plan's count bounded by one partly filled
// group per instance
static inline int64_t em_groups(const EmMfmaArgs &a, int mw)
{
    const int64_t full = (a.B + mw - 1) / mw;
    return a.inst ? full + a.P : full;
}

// Workgroup plan of a batch: the instances in decreasing order of windows
// (the longest sweeps start first), each cut into groups of 16 kWaves G
// consecutive buckets (the models of one workgroup).  Layout: wg_start[P + 1] (first workgroup of each rank),
// b0[P], b1[P] (bucket range of each instance), order[P] (instance of each rank).
struct PlanView {
    const int64_t *wg_start, *b0, *b1, *order;
};
__host__ __device__ inline PlanView plan_view(const int64_t *plan, int P)
{
    return PlanView{plan, plan + P + 1, plan + 2 * P + 1, plan + 3 * P + 1};
}

constexpr int kWaves = 4;  // waves (groups of 16 models) per workgroup
// tile shape 10 G + PPB: G groups of 16 models per wave, PPB window pairs
// built per workgroup barrier
constexpr int kShapeDefault = 14;  // untuned
constexpr int kMaxMT2 = 6;         // G = 2 for ceil(l/4) <= 6 (registers)
constexpr float kPOff = 3.0f;
constexpr float kSlack = 12.0f;

// 32 DNA symbols starting at P (MSB-first) as hi (P..P+15) and lo (P+16..P+31).
// CLAMP: reads clamped below nw (global memory); otherwise the buffer is padded.
template <bool CLAMP>
__device__ __forceinline__ void dna32(const uint32_t *w, int64_t P, int64_t nw, uint32_t &hi, uint32_t &lo)
{
    const int64_t wi = P >> 4;
    const uint32_t r = (uint32_t)(P & 15) << 1;
    uint32_t w0, w1, w2;
    if (CLAMP) {
        w0 = w[wi < nw ? wi : nw - 1];
        w1 = w[wi + 1 < nw ? wi + 1 : nw - 1];
        w2 = w[wi + 2 < nw ? wi + 2 : nw - 1];
    } else {
        w0 = w[wi];
        w1 = w[wi + 1];
        w2 = w[wi + 2];
    }
    hi = (uint32_t)((((uint64_t)w0 << 32) | w1) >> (32 - r));
    lo = (uint32_t)((((uint64_t)w1 << 32) | w2) >> (32 - r));
}

// where a workgroup's one-hot tables come from
constexpr int kSrcGlobal = 0;  // built in the kernel from the packed instance (no workspace)
constexpr int kSrcPre = 2;     // copied from tables precomputed once per call (k_em_tables)

// Precomputed tables: pair j (windows 32j .. 32j+31) of sequence i of an
// instance sits in slot i + floor(W_i / 32) + j, W_i = offsets[i] - i (l - 1)
// being the sequence's first window in the instance's window numbering.  A
// sequence of L_i windows ends at slot i + floor((W_i + L_i) / 32) at most, so
// the slots of different sequences never overlap and an instance needs at
// most t + ceil(x / 32) of them (a few stay unused).
__host__ __device__ inline int64_t em_inst_slots(int64_t t, int64_t x) { return t + (x + 31) / 32; }

__device__ __forceinline__ int64_t seq_slot0(const int64_t *offsets, int i, int l)
{
    return i + (offsets[i] - (int64_t)i * (l - 1)) / 32;
}

// fp16(p - hi) for two values whose fp16 roundings are packed in hi2
__device__ __forceinline__ uint32_t split_lo(uint32_t hi2, float p0, float p1)
{
    uint32_t r;
    asm volatile(
        "v_fma_mixlo_f16 %0, %1, -1.0, %2 op_sel_hi:[1,0,0]\n\t"
        "v_fma_mixhi_f16 %0, %1, -1.0, %3 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
        : "=&v"(r)
        : "v"(hi2), "v"(p0), "v"(p1));
    return r;
}

__device__ __forceinline__ uint32_t pack_hi(float p0, float p1)
{
    return __builtin_bit_cast(uint32_t, half2v{(_Float16)p0, (_Float16)p1});
}

// E-step k-blocks (8 positions each) for MT M-tiles (4 positions each)
template <int MT>
struct Tiles {
    static constexpr int LB = (MT + 1) / 2;
    static constexpr int CX = 4 * MT;       // count rows (positions) of a model
    static constexpr int NE = 4 * MT + 12;  // M-step table entries a pair reads
};

// Split form with an odd number of 4-position tiles: the last k-block holds
// at most four real positions, so its hi and lo halves share one MFMA (lane
// groups 0, 1 carry the hi halves of its positions, groups 2, 3 the lo halves
// of the same positions) instead of two MFMAs each half zero.
template <int MT, bool SPLIT>
constexpr bool kMergeTail = SPLIT && (MT & 1) != 0;

// one-hot tables of one window pair: the symbols at s0 + a0 + e
template <int MT>
struct alignas(16) PairTables {
    uint32_t oh2[64][4];          // letters 0..3 of symbol e, then of symbol e+1
    uint4 mt8[Tiles<MT>::NE][4];  // [e][c]: symbols e..e+3 and e+16..e+19 == c
};
// 16-byte quads of one pair's tables: at most 256, one per thread of a workgroup
template <int MT>
constexpr int kTabQuads = (int)(sizeof(PairTables<MT>) / 16);
static_assert(kTabQuads<8> <= 256, "one quad per thread");

// lut[y]: four FP16 halves, half q = 1.0 where 2-bit field q of y (from the top)
// is zero.  With y = (4 symbols) ^ (c * 0x55) that is the one-hot of letter c.
__device__ __forceinline__ void build_lut(uint2 *lut)
{
    const uint32_t y = threadIdx.x;  // the workgroup has 256 threads
    uint32_t h[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) h[q] = ((y >> (6 - 2 * q)) & 3u) ? 0u : 0x3C00u;
    lut[y] = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
}

// Workgroup-cooperative build: thread (e = tid / 4, c = tid % 4) writes
// mt8[e][c] (e < NE) and word c of oh2[e].
template <int MT, bool CLAMP>
__device__ __forceinline__ void build_tables(const uint32_t *W, int64_t nw, int64_t base, const uint2 *lut,
                                             PairTables<MT> &T)
{
    const int tid = threadIdx.x, e = tid >> 2;
    const uint32_t c = tid & 3u;
    uint32_t hi, lo;
    dna32<CLAMP>(W, base + e, nw, hi, lo);
    if (e < Tiles<MT>::NE) {
        const uint32_t cc = c * 0x55u;
        const uint2 u0 = lut[(hi >> 24) ^ cc], u1 = lut[(lo >> 24) ^ cc];
        T.mt8[e][c] = make_uint4(u0.x, u0.y, u1.x, u1.y);
    }
    // word c of oh2[e]: letters 2(c&1), 2(c&1)+1 of symbol e (c < 2) or e+1
    const uint32_t sym = c < 2 ? hi >> 30 : (hi >> 28) & 3u;
    T.oh2[e][c] = (sym >> 1) == (c & 1u) ? 0x3C00u << ((sym & 1u) << 4) : 0u;
}

struct SeqState {
    float4v neg;  // kPOff - mref in every component: the E-step accumulators' start
    float mref;   // reference (log2 units) of the scores
    double srun;  // this lane's share of sum 2^(S - mref + kPOff), in FP64
    float bestv;  // final E-step: best score and window of this lane
    int besti;
};

// One pair of 16-window tiles (windows a0 .. a0+31 of one sequence) for this
// wave's G groups of 16 models; the groups share the A operands.
// LDS byte offsets of this lane's fragments within a pair's tables, formed
// once per kernel: E-step A (positions 2g, 2g+1 of window r), the same for a
// merged last k-block (positions 2(g & 1), 2(g & 1)+1), M-step A
struct FragOff {
    uint32_t a, a_merged, m;
};

template <int MT, bool LAST, bool TAIL, bool SPLIT, int G>
__device__ __forceinline__ void tile_pair(int a0, int L, const PairTables<MT> &T, const FragOff &fo,
                                          const half8 (&Whi)[G][Tiles<MT>::LB],
                                          const half8 (&Wlo)[G][Tiles<MT>::LB], float4v (&O)[G][MT],
                                          SeqState (&st)[G])
{
    constexpr int LB = Tiles<MT>::LB;
    constexpr bool MERGE = kMergeTail<MT, SPLIT>;
    const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
    const char *tb = reinterpret_cast<const char *>(&T);
    half8 Ae[2][LB];
#pragma unroll
    for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
        for (int kb = 0; kb < LB; ++kb) {
            // entry 16 t2 + 8 kb + (r + 2g) of oh2 (16 B each); a merged last
            // block's groups 2, 3 repeat the positions of groups 0, 1
            const uint32_t off = MERGE && kb == LB - 1 ? fo.a_merged : fo.a;
            Ae[t2][kb] = *reinterpret_cast<const half8 *>(tb + off + (16 * t2 + 8 * kb) * 16);
        }
    // E-step, already shifted: S' = S - (mref - kPOff); one chain per tile and group
    float4v S0[G], S1[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
        S0[q] = st[q].neg;
        S1[q] = st[q].neg;
    }
#pragma unroll
    for (int kb = 0; kb < LB; ++kb)
#pragma unroll
        for (int q = 0; q < G; ++q) {
            S0[q] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Ae[0][kb], Whi[q][kb], S0[q], 0, 0, 0);
            S1[q] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Ae[1][kb], Whi[q][kb], S1[q], 0, 0, 0);
            if (SPLIT && !(MERGE && kb == LB - 1)) {
                S0[q] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Ae[0][kb], Wlo[q][kb], S0[q], 0, 0, 0);
                S1[q] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Ae[1][kb], Wlo[q][kb], S1[q], 0, 0, 0);
            }
        }
    half8 Am[MT];
    if (!LAST) {
        // M-step A operand: row (position pm, letter cm); windows 4g..4g+3 of both tiles
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)  // mt8[4g + 4mt + r/4][r % 4]
            Am[mt] = *reinterpret_cast<const half8 *>(tb + fo.m + mt * 256);
    }
#pragma unroll
    for (int q = 0; q < G; ++q) {
        float S[8];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            S[j] = S0[q][j];
            S[4 + j] = S1[q][j];
        }
        if (TAIL) {
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (a0 + 16 * (u >> 2) + 4 * g + (u & 3) >= L) S[u] = -INFINITY;
        }
        // the common path needs only whether a score passed the slack, not the
        // maximum (which fmaxf would form after quieting each operand)
        bool big = false;
#pragma unroll
        for (int u = 0; u < 8; ++u) big |= S[u] > kPOff + kSlack;
        if (LAST) {
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (S[u] - st[q].neg[0] > st[q].bestv) {
                    st[q].bestv = S[u] - st[q].neg[0];
                    st[q].besti = a0 + 16 * (u >> 2) + 4 * g + (u & 3);
                }
        }
        if (__builtin_expect(__ballot(big) != 0, 0)) {
            // rare: move the reference up to the model's new maximum
            float tm = fmaxf(fmaxf(fmaxf(S[0], S[1]), fmaxf(S[2], S[3])), fmaxf(fmaxf(S[4], S[5]), fmaxf(S[6], S[7])));
            tm = fmaxf(tm, __shfl_xor(tm, 16));
            tm = fmaxf(tm, __shfl_xor(tm, 32));
            // a whole number of binades, so that the rescales below are exact
            const float d = tm > kPOff + kSlack ? ceilf(tm - kPOff) : 0.f;
            const float al = __builtin_amdgcn_exp2f(-d);
            st[q].srun *= (double)al;
            if (!LAST)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) O[q][mt] *= al;
#pragma unroll
            for (int u = 0; u < 8; ++u) S[u] -= d;
            st[q].mref += d;
            const float n = kPOff - st[q].mref;  // exactly what the scores are shifted by
            st[q].neg = float4v{n, n, n, n};
        }
        float P[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) P[u] = __builtin_amdgcn_exp2f(S[u]);
        // the lane's eight terms of this pair (a three-level FP32 tree, relative
        // error at most 3 * 2^-24), accumulated over the sequence in FP64
        st[q].srun += (double)(((P[0] + P[1]) + (P[2] + P[3])) + ((P[4] + P[5]) + (P[6] + P[7])));
        if (!LAST) {
            uint4 h;
            h.x = pack_hi(P[0], P[1]);
            h.y = pack_hi(P[2], P[3]);
            h.z = pack_hi(P[4], P[5]);
            h.w = pack_hi(P[6], P[7]);
            const half8 Ph = __builtin_bit_cast(half8, h);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                O[q][mt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Am[mt], Ph, O[q][mt], 0, 0, 0);
            if (SPLIT) {
                uint4 lw;
                lw.x = split_lo(h.x, P[0], P[1]);
                lw.y = split_lo(h.y, P[2], P[3]);
                lw.z = split_lo(h.z, P[4], P[5]);
                lw.w = split_lo(h.w, P[6], P[7]);
                const half8 Pl = __builtin_bit_cast(half8, lw);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    O[q][mt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Am[mt], Pl, O[q][mt], 0, 0, 0);
            }
        }
    }
}

// This thread's quads of the tables of the PPB window pairs starting at
// window a0 of sequence i (kSrcPre): loaded into registers one step ahead of
// their use, written to LDS at the step that uses them.
template <int MT, int PPB>
__device__ __forceinline__ void fetch_tables(const EmMfmaArgs &a, int64_t slot0, int L, int a0, u32x4 (&pf)[PPB])
{
    // every load is unconditional and in bounds (a pair past the sequence's
    // end re-reads the step's first pair, threads past the quads re-read the
    // last one), which keeps pf in registers; only the LDS writes are guarded
    constexpr int NQ = kTabQuads<MT>;
    const int q = (int)threadIdx.x < NQ ? (int)threadIdx.x : NQ - 1;
    const u32x4 *src = reinterpret_cast<const u32x4 *>(a.tables) + (slot0 + a0 / 32) * NQ + q;
#pragma unroll
    for (int u = 0; u < PPB; ++u) pf[u] = src[(a0 + 32 * u < L ? u : 0) * NQ];
}

// windows and first table slot of sequence i of the instance whose first slot
// is tb (kSrcPre)
__device__ __forceinline__ void seq_slots(const EmMfmaArgs &a, int64_t tb, int i, int &L, int64_t &slot0)
{
    L = (int)(a.offsets[i + 1] - a.offsets[i]) - a.l + 1;
    slot0 = tb + seq_slot0(a.offsets, i, a.l);
}

// One sequence: every window pair (tables built by the whole workgroup, or
// copied from the precomputed ones), then the per-sequence log-sum-exp and
// counts, or, in the final E-step, the best start of every model.  acc[q]:
// the count accumulators of group q.  kSrcPre: pf holds this thread's quads of
// the sequence's first step on entry and of the step after the sequence (the
// next sequence's first, or sequence 0's for the next iteration) on return.
template <int MT, int SRC, bool LAST, bool SPLIT, int PPB, int G>
__device__ __forceinline__ void sweep(const EmMfmaArgs &a, const uint32_t *W, const uint2 *lut, int i, int64_t bw,
                                      int64_t nvalid, PairTables<MT> *tabs, int &parity, int64_t tb,
                                      u32x4 (&pf)[PPB], float (*acc)[16][Tiles<MT>::CX][4],
                                      const half8 (&Whi)[G][Tiles<MT>::LB], const half8 (&Wlo)[G][Tiles<MT>::LB],
                                      const float (&mlow)[G], double (&llr)[G])
{
    const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
    const int64_t s0 = a.offsets[i];
    const int L = (int)(a.offsets[i + 1] - s0) - a.l + 1;
    static_assert(offsetof(PairTables<MT>, mt8) == 1024, "M-step fragments follow the 1 KB of E-step ones");
    const FragOff fo{(uint32_t)(r + 2 * g) * 16u, (uint32_t)(r + 2 * (g & 1)) * 16u,
                     1024u + (uint32_t)((4 * g + (r >> 2)) * 4 + (r & 3)) * 16u};
    // kSrcPre: this sequence's first slot and the next sequence's size and
    // first slot, formed once here rather than at every step
    int64_t sl = 0, sln = 0;
    int Ln = 0;
    if constexpr (SRC == kSrcPre) {
        int Li;
        seq_slots(a, tb, i, Li, sl);
        seq_slots(a, tb, i + 1 < a.t ? i + 1 : 0, Ln, sln);
    }
    float4v O[G][MT];
    SeqState st[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) O[q][mt] = float4v{0.f, 0.f, 0.f, 0.f};
        // the reference starts at the lowest score the model can give
        const float n0 = kPOff - mlow[q];
        st[q] = SeqState{float4v{n0, n0, n0, n0}, mlow[q], 0.0, -INFINITY, 0};
    }
    for (int a0 = 0; a0 < L; a0 += 32 * PPB) {
        PairTables<MT> *T = tabs + PPB * parity;
        parity ^= 1;
        if constexpr (SRC == kSrcPre) {
#pragma unroll
            for (int u = 0; u < PPB; ++u)
                if (a0 + 32 * u < L && threadIdx.x < kTabQuads<MT>)
                    reinterpret_cast<u32x4 *>(&T[u])[threadIdx.x] = pf[u];
        } else {
#pragma unroll
            for (int u = 0; u < PPB; ++u)
                if (a0 + 32 * u < L) build_tables<MT, SRC == kSrcGlobal>(W, a.nwords, s0 + a0 + 32 * u, lut, T[u]);
        }
        __syncthreads();
        if constexpr (SRC == kSrcPre) {
            // the next step's quads (this sequence's, or the next sequence's
            // first) load while this step computes
            const int na = a0 + 32 * PPB;
            if (na < L) fetch_tables<MT, PPB>(a, sl, L, na, pf);
            else fetch_tables<MT, PPB>(a, sln, Ln, 0, pf);
        }
#pragma unroll
        for (int u = 0; u < PPB; ++u) {
            const int b0 = a0 + 32 * u;
            if (b0 + 32 <= L) tile_pair<MT, LAST, false, SPLIT, G>(b0, L, T[u], fo, Whi, Wlo, O, st);
            else if (b0 < L) tile_pair<MT, LAST, true, SPLIT, G>(b0, L, T[u], fo, Whi, Wlo, O, st);
        }
    }
#pragma unroll
    for (int q = 0; q < G; ++q) {
        // the model's sum over the sequence's windows: the four lane groups'
        // FP64 partials combined in FP64
        double sr = st[q].srun;
        sr += __shfl_xor(sr, 16);
        sr += __shfl_xor(sr, 32);
        const double ln2 = 0.6931471805599453;
        const double lse = ((double)st[q].mref - (double)kPOff) * ln2 + log(sr);
        llr[q] += lse - log((double)L);
        if (!LAST) {
            const float inv = (float)(1.0 / sr);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                float4v *dst = reinterpret_cast<float4v *>(&acc[q][r][4 * mt + g][0]);
                *dst += O[q][mt] * inv;
            }
        } else if (a.sites) {
            float bv = st[q].bestv;
            int bi = st[q].besti;
#pragma unroll
            for (int o = 16; o <= 32; o <<= 1) {
                const float ov = __shfl_xor(bv, o);
                const int oi = __shfl_xor(bi, o);
                if (ov > bv || (ov == bv && oi < bi)) {
                    bv = ov;
                    bi = oi;
                }
            }
            const int64_t b = bw + 16 * q + r;
            if (g == 0 && b < nvalid) a.sites[b * a.site_stride + i] = bi;
        }
    }
}

// static LDS of a workgroup and the waves per SIMD to compile for: three when
// the registers of ceil(l/4) <= 5 allow it and three workgroups' LDS (with 6 KB
// of headroom each) fit the 160 KB of a CU, else two
template <int MT, int PPB, int G>
constexpr int em_static_lds()
{
    return 2 * PPB * (int)sizeof(PairTables<MT>) + 256 * (int)sizeof(uint2) + kWaves * G * 16 * Tiles<MT>::CX * 16;
}
template <int MT, int PPB, int G>
constexpr int em_waves_per_simd()
{
    return MT <= 5 && 3 * (em_static_lds<MT, PPB, G>() + 6 * 1024) <= 160 * 1024 ? 3 : 2;
}

// G groups of 16 models per wave, kWaves waves per workgroup
template <int MT, int SRC, bool SPLIT, int PPB, int G>
__global__ void __launch_bounds__(64 * kWaves, (em_waves_per_simd<MT, PPB, G>())) k_em_mfma(const EmMfmaArgs a0)
{
    constexpr int LB = Tiles<MT>::LB, CX = Tiles<MT>::CX, MW = 16 * kWaves * G;
    __shared__ __align__(16) PairTables<MT> tabs[2 * PPB];
    __shared__ __align__(16) uint2 lut[256];
    __shared__ __align__(16) float accs[kWaves][G][16][CX][4];
    __shared__ float lbg2[4];  // log2 bg[c], formed once for every iteration's log-odds

    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
    EmMfmaArgs a = a0;
    int64_t b0, nvalid, tb = 0;
    if (a0.inst) {
        // batch: find this workgroup's instance rank, largest r with wg_start[r] <= wg
        const PlanView pv = plan_view(a0.plan, a0.P);
        const int64_t wg = blockIdx.x;
        if (wg >= pv.wg_start[a0.P]) return;
        int lo = 0, hi = a0.P;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (pv.wg_start[mid] <= wg) lo = mid;
            else hi = mid;
        }
        const int p = (int)pv.order[lo];
        const pm_inst I = a0.inst[p];
        a.packed = I.packed;
        a.offsets = I.offsets;
        a.t = I.t;
        a.nwords = (I.n_total + 15) / 16 + 4;
        tb = a0.tbase ? a0.tbase[p] : 0;
        b0 = pv.b0[p] + (wg - pv.wg_start[lo]) * MW;
        nvalid = pv.b1[p] < b0 + MW ? pv.b1[p] : b0 + MW;
    } else {
        nvalid = a.n_dev ? *a.n_dev : a.B;
        if (nvalid > a.B) nvalid = a.B;
        b0 = (int64_t)blockIdx.x * MW;
        if (b0 >= nvalid) return;  // uniform over the workgroup
    }
    const uint32_t *W = a.packed;
    const uint2 *lutp = nullptr;
    u32x4 pf[PPB];
    if constexpr (SRC == kSrcPre) {
        int L0;
        int64_t sl0;
        seq_slots(a, tb, 0, L0, sl0);
        fetch_tables<MT, PPB>(a, sl0, L0, 0, pf);  // the first step of the first sweep
    } else {
        build_lut(lut);
        lutp = lut;
    }
    // by the same FP32 logarithm as the models' log2 theta, so that theta = bg
    // gives log-odds of exactly zero
    if (threadIdx.x < 4) lbg2[threadIdx.x] = __builtin_amdgcn_logf((float)a.bg[threadIdx.x]);
    __syncthreads();
    const int64_t bw = b0 + 16 * G * wv;
    float (*acc)[16][CX][4] = accs[wv];
    const int l = a.l, t = a.t, AL = 4 * l;
    const double beta = a.beta;
    int parity = 0;

    half8 Whi[G][LB], Wlo[G][LB];
    for (int it = 0; it <= a.iters; ++it) {
        const bool last = it == a.iters;
        const double *src = it == 0 ? a.theta0 : a.theta_out;
        // ---- log-odds (log2 units) of the lane's E-step B operands: model r of
        // group q, positions 8kb+2g and 8kb+2g+1, letters 0..3, split in two
        // FP16 halves (a merged last block: hi halves in groups 0, 1, lo halves
        // of the same positions in groups 2, 3); the lane's hi entries cover
        // every position once across the four lane groups, so the prior and the
        // lowest score are lane sums over them
        double prior[G];
        float mlow[G];
        // the lane's position base goes through an empty asm statement so that
        // the index arithmetic below is formed here each iteration rather than
        // hoisted out of the loop into registers the sweeps need
        int g2 = 2 * g;
        asm volatile("" : "+v"(g2));
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const int64_t b = bw + 16 * q + r;
            const bool vb = b < nvalid;
            double pr = 0;
            float wmin = 0.f;
#pragma unroll
            for (int kb = 0; kb < LB; ++kb) {
                const bool lo_half = kMergeTail<MT, SPLIT> && kb == LB - 1 && g2 >= 4;
                half8 hi, lo;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int p = 8 * kb + (lo_half ? g2 - 4 : g2) + h;
                    float mn = 0.f;
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        float w = 0.f;
                        if (p < l && vb) {
                            const double th = src[b * AL + c * l + p];
                            if (it == 0 && !lo_half) a.theta_out[b * AL + c * l + p] = th;
                            // log2 theta by the hardware FP32 logarithm (about 2^-23
                            // relative, within what the split FP16 halves carry)
                            const float l2 = __builtin_amdgcn_logf((float)th);
                            w = l2 - lbg2[c];
                            if (!lo_half) pr += a.bg[c] * (double)l2;  // log2 units
                        }
                        mn = c == 0 ? w : fminf(mn, w);
                        hi[4 * h + c] = (_Float16)w;
                        lo[4 * h + c] = (_Float16)(w - (float)hi[4 * h + c]);
                    }
                    if (!lo_half) wmin += mn;
                }
                Whi[q][kb] = lo_half ? lo : hi;
                Wlo[q][kb] = lo;
            }
            pr += __shfl_xor(pr, 16);
            pr += __shfl_xor(pr, 32);
            wmin += __shfl_xor(wmin, 16);
            wmin += __shfl_xor(wmin, 32);
            prior[q] = pr * 0.6931471805599453;  // natural log
            // lowest possible score, a little below to absorb rounding
            mlow[q] = wmin - 1.0f;
        }
        // ---- clear the count accumulators (own entries)
#pragma unroll
        for (int q = 0; q < G; ++q)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                *reinterpret_cast<float4v *>(&acc[q][r][4 * mt + g][0]) = float4v{0.f, 0.f, 0.f, 0.f};
        __syncthreads();  // tables free

        double llr[G];
#pragma unroll
        for (int q = 0; q < G; ++q) llr[q] = 0;
        for (int i = 0; i < t; ++i) {
            if (last)
                sweep<MT, SRC, true, SPLIT, PPB, G>(a, W, lutp, i, bw, nvalid, tabs, parity, tb, pf, acc, Whi, Wlo,
                                                    mlow, llr);
            else
                sweep<MT, SRC, false, SPLIT, PPB, G>(a, W, lutp, i, bw, nvalid, tabs, parity, tb, pf, acc, Whi, Wlo,
                                                     mlow, llr);
        }
        // ---- objective of theta^it, then the M-step (own entries)
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const int64_t b = bw + 16 * q + r;
            const bool vb = b < nvalid;
            if (g == 0 && vb) {
                a.J[b * (a.iters + 1) + it] = llr[q] + beta * prior[q];
                if (a.llr) a.llr[b * (a.iters + 1) + it] = llr[q];
            }
            if (!last && vb) {
                #pragma unroll 1
                for (int mt = 0; mt < MT; ++mt) {
                    const int p = 4 * mt + g;
                    if (p < l) {
                        const float4v cn = *reinterpret_cast<const float4v *>(&acc[q][r][p][0]);
                        // every column's counts sum to t: normalising by the column's
                        // own total is the same update and stays on the simplex
                        const double tot = (double)cn[0] + (double)cn[1] + (double)cn[2] + (double)cn[3] + beta;
                        #pragma unroll 1
                        for (int c = 0; c < 4; ++c)
                            a.theta_out[b * AL + c * l + p] = ((double)cn[c] + beta * a.bg[c]) / tot;
                    }
                }
            }
        }
        // theta^(it+1) visible to the lanes that read it: a lane's log-odds
        // entries were normalised by other lanes of its wave
        __syncthreads();
    }
}

// One workgroup per table slot: the one-hot tables of one window pair in the
// layout the EM kernel copies into LDS.  Batch: the slot's instance from
// tbase (first slot of every instance, ascending).  Slots past a sequence's
// last pair are left untouched; nothing reads them.
struct EmTabArgs {
    pm_inst one;           // the instance when inst is NULL
    const pm_inst *inst;   // batch instance table, or NULL
    const int64_t *tbase;  // batch: [P + 1]
    int P, l;
    int64_t nslots;        // slots of the launch
    int64_t nwords_one;    // packed words of `one` (reads are clamped below)
    uint8_t *tables;
};

template <int MT>
__global__ void __launch_bounds__(256) k_em_tables(const EmTabArgs a)
{
    __shared__ __align__(16) uint2 lut[256];
    const int64_t slot = blockIdx.x;
    if (slot >= a.nslots) return;
    pm_inst I = a.one;
    int64_t rel = slot, nw = a.nwords_one;
    if (a.inst) {
        if (slot >= a.tbase[a.P]) return;
        int lo = 0, hi = a.P;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (a.tbase[mid] <= slot) lo = mid;
            else hi = mid;
        }
        I = a.inst[lo];
        rel = slot - a.tbase[lo];
        nw = (I.n_total + 15) / 16 + 4;
    }
    // the sequence: largest i with seq_slot0(i) <= rel (seq_slot0 increases with i)
    int lo = 0, hi = I.t;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (seq_slot0(I.offsets, mid, a.l) <= rel) lo = mid;
        else hi = mid;
    }
    const int64_t j = rel - seq_slot0(I.offsets, lo, a.l);
    const int64_t s0 = I.offsets[lo];
    const int L = (int)(I.offsets[lo + 1] - s0) - a.l + 1;
    if (32 * j >= L) return;  // uniform over the workgroup
    build_lut(lut);
    __syncthreads();
    build_tables<MT, true>(I.packed, nw, s0 + 32 * j, lut, reinterpret_cast<PairTables<MT> *>(a.tables)[slot]);
}

static size_t pair_table_bytes(int mt) { return 1024 + (size_t)(4 * mt + 12) * 64; }
static_assert(sizeof(PairTables<1>) == 1024 + 16 * 64 && sizeof(PairTables<8>) == 1024 + 44 * 64, "table size");

static int launch_em_tables(const EmTabArgs &t, hipStream_t st)
{
    if (t.nslots < 1) return PM_OK;
    switch ((t.l + 3) / 4) {
    case 1: hipLaunchKernelGGL(k_em_tables<1>, dim3((unsigned)t.nslots), dim3(256), 0, st, t); break;
    case 2: hipLaunchKernelGGL(k_em_tables<2>, dim3((unsigned)t.nslots), dim3(256), 0, st, t); break;
    case 3: hipLaunchKernelGGL(k_em_tables<3>, dim3((unsigned)t.nslots), dim3(256), 0, st, t); break;
    case 4: hipLaunchKernelGGL(k_em_tables<4>, dim3((unsigned)t.nslots), dim3(256), 0, st, t); break;
    case 5: hipLaunchKernelGGL(k_em_tables<5>, dim3((unsigned)t.nslots), dim3(256), 0, st, t); break;
    case 6: hipLaunchKernelGGL(k_em_tables<6>, dim3((unsigned)t.nslots), dim3(256), 0, st, t); break;
    case 7: hipLaunchKernelGGL(k_em_tables<7>, dim3((unsigned)t.nslots), dim3(256), 0, st, t); break;
    default: hipLaunchKernelGGL(k_em_tables<8>, dim3((unsigned)t.nslots), dim3(256), 0, st, t); break;
    }
    PM_LAUNCHED();
    return PM_OK;
}

static int64_t seqs_slots(const pm_seqs *S, int l) { return em_inst_slots(S->t, S->n_total - (int64_t)S->t * (l - 1)); }

size_t em_tables_workspace(const pm_seqs *S, int32_t l)
{
    return (size_t)seqs_slots(S, l) * pair_table_bytes((l + 3) / 4);
}

// precomputed tables of one instance into ws (checked size), a.tables set
static int prepare_tables(EmMfmaArgs &a, const pm_seqs *S, int l, void *ws, size_t ws_bytes, hipStream_t st)
{
    a.tables = nullptr;
    if (!ws) return PM_OK;
    const size_t need = em_tables_workspace(S, l);
    if (ws_bytes < need) return fail(PM_EINVAL, "workspace of %zu bytes, the one-hot tables need %zu", ws_bytes, need);
    if (((uintptr_t)ws & 15) != 0) return fail(PM_EINVAL, "workspace must be 16-byte aligned");
    EmTabArgs t{};
    t.one.offsets = S->offsets;
    t.one.packed = S->packed;
    t.one.n_total = S->n_total;
    t.one.t = S->t;
    t.l = l;
    t.nslots = seqs_slots(S, l);
    t.nwords_one = pm_packed_words(S->alphabet, S->n_total);
    t.tables = static_cast<uint8_t *>(ws);
    const int rc = launch_em_tables(t, st);
    if (rc != PM_OK) return rc;
    a.tables = t.tables;
    return PM_OK;
}

template <int MT, bool SPLIT, int PPB, int G>
static int launch_em_mfma(const EmMfmaArgs &a, hipStream_t st)
{
    const int64_t groups = em_groups(a, 16 * kWaves * G);
    if (a.tables)
        hipLaunchKernelGGL((k_em_mfma<MT, kSrcPre, SPLIT, PPB, G>), dim3((unsigned)groups), dim3(64 * kWaves), 0, st,
                           a);
    else
        hipLaunchKernelGGL((k_em_mfma<MT, kSrcGlobal, SPLIT, PPB, G>), dim3((unsigned)groups), dim3(64 * kWaves), 0,
                           st, a);
    PM_LAUNCHED();
    return PM_OK;
}

// tile shape in use per (ceil(l/4) - 1, split), coded 10 G + PPB; 0 = untuned
static int g_shape[8][2];

static bool shape_ok(int shape, int l)
{
    const int G = shape / 10, ppb = shape % 10;
    return (ppb == 1 || ppb == 2 || ppb == 4) && (G == 1 || (G == 2 && (l + 3) / 4 <= kMaxMT2));
}

static int tuned_shape(int l, bool split)
{
    const int v = g_shape[(l + 3) / 4 - 1][split ? 1 : 0];
    return v ? v : kShapeDefault;
}

template <bool SPLIT, int PPB, int G>
static int dispatch_mt(const EmMfmaArgs &a, hipStream_t st)
{
    switch ((a.l + 3) / 4) {
    case 1: return launch_em_mfma<1, SPLIT, PPB, G>(a, st);
    case 2: return launch_em_mfma<2, SPLIT, PPB, G>(a, st);
    case 3: return launch_em_mfma<3, SPLIT, PPB, G>(a, st);
    case 4: return launch_em_mfma<4, SPLIT, PPB, G>(a, st);
    case 5: return launch_em_mfma<5, SPLIT, PPB, G>(a, st);
    case 6: return launch_em_mfma<6, SPLIT, PPB, G>(a, st);
    case 7: if (G == 1) return launch_em_mfma<7, SPLIT, PPB, 1>(a, st); break;
    default: if (G == 1) return launch_em_mfma<8, SPLIT, PPB, 1>(a, st); break;
    }
    return fail(PM_EINVAL, "tile shape with %d model groups per wave needs l <= %d", G, 4 * kMaxMT2);
}

template <bool SPLIT>
static int dispatch_shape(const EmMfmaArgs &a, hipStream_t st, int shape)
{
    switch (shape) {
    case 11: return dispatch_mt<SPLIT, 1, 1>(a, st);
    case 12: return dispatch_mt<SPLIT, 2, 1>(a, st);
    case 14: return dispatch_mt<SPLIT, 4, 1>(a, st);
    case 21: return dispatch_mt<SPLIT, 1, 2>(a, st);
    case 22: return dispatch_mt<SPLIT, 2, 2>(a, st);
    default: return dispatch_mt<SPLIT, 4, 2>(a, st);
    }
}

// shape 0: the one recorded for this length class and precision
static int dispatch_em_mfma(const EmMfmaArgs &a, hipStream_t st, int shape = 0)
{
    if (!shape) shape = tuned_shape(a.l, a.split != 0);
    if (!shape_ok(shape, a.l)) shape = 10 + shape % 10;
    return a.split ? dispatch_shape<true>(a, st, shape) : dispatch_shape<false>(a, st, shape);
}

int em_refine_mfma(const pm_seqs *S, int32_t l, const double *theta0, const double *bg, int64_t B,
                   const int64_t *n_dev, int32_t iters, double beta, double *theta_out, double *J_out,
                   double *llr_out, int32_t *sites_out, void *ws, size_t ws_bytes, bool split, hipStream_t st)
{
    EmMfmaArgs a{};
    a.split = split;
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
    a.site_stride = S->t;
    a.l = l;
    a.iters = iters;
    a.beta = beta;
    const int rc = prepare_tables(a, S, l, ws, ws_bytes, st);
    if (rc != PM_OK) return rc;
    return dispatch_em_mfma(a, st);
}

// One workgroup: each instance's bucket range (buckets ascend by item), its
// workgroup count, the largest-first order of the instances and the scan of
// the counts in that order.
__global__ void __launch_bounds__(1024) k_em_plan(const pm_inst *inst, int P, const pm_bucket *buckets,
                                                 const int64_t *n_dev, int64_t Bcap, int mw, int64_t *plan,
                                                 int64_t *tbase)
{
    const PlanView pv = plan_view(plan, P);
    int64_t *wg_start = const_cast<int64_t *>(pv.wg_start), *b0 = const_cast<int64_t *>(pv.b0);
    int64_t *b1 = const_cast<int64_t *>(pv.b1), *order = const_cast<int64_t *>(pv.order);
    int64_t nvalid = n_dev ? *n_dev : Bcap;
    if (nvalid > Bcap) nvalid = Bcap;
    // bucket range of every instance: first bucket whose item is >= first_item
    for (int p = threadIdx.x; p < P; p += 1024) {
        for (int side = 0; side < 2; ++side) {
            const int64_t item = (int64_t)inst[p].first_item + (side ? inst[p].m : 0);
            int64_t lo = 0, hi = nvalid;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if ((int64_t)buckets[mid].trial < item) lo = mid + 1;
                else hi = mid;
            }
            (side ? b1 : b0)[p] = lo;
        }
    }
    // rank by windows, descending, ties by index
    for (int p = threadIdx.x; p < P; p += 1024) {
        const int64_t xp = inst[p].x;
        int r = 0;
        for (int q = 0; q < P; ++q) {
            const int64_t xq = inst[q].x;
            r += (xq > xp || (xq == xp && q < p)) ? 1 : 0;
        }
        order[r] = p;
    }
    __syncthreads();
    // exclusive scan of the workgroup counts in rank order (serial: P is small)
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int r = 0; r < P; ++r) {
            wg_start[r] = run;
            const int p = (int)order[r];
            run += (b1[p] - b0[p] + mw - 1) / mw;
        }
        wg_start[P] = run;
        // first precomputed-table slot of every instance, in instance order
        if (tbase) {
            int64_t sl = 0;
            for (int p = 0; p < P; ++p) {
                tbase[p] = sl;
                sl += em_inst_slots(inst[p].t, inst[p].x);
            }
            tbase[P] = sl;
        }
    }
}

// batch workspace: the plan, the instances' first table slots, the tables
static size_t plan_bytes(int32_t P) { return ((size_t)(4 * (int64_t)P + 1) * sizeof(int64_t) + 255) / 256 * 256; }
static size_t tbase_bytes(int32_t P) { return ((size_t)(P + 1) * sizeof(int64_t) + 255) / 256 * 256; }
static int64_t batch_slots(const pm_batch *Bt)
{
    int64_t sl = 0;
    for (int p = 0; p < Bt->P; ++p) sl += em_inst_slots(Bt->inst_host[p].t, Bt->inst_host[p].x);
    return sl;
}

size_t em_batch_workspace(const pm_batch *Bt, bool tables)
{
    if (Bt->P < 1) return 0;
    size_t n = plan_bytes(Bt->P) + tbase_bytes(Bt->P);
    if (tables) n += (size_t)batch_slots(Bt) * pair_table_bytes((Bt->l + 3) / 4);
    return n;
}

int em_refine_mfma_batch(const pm_batch *Bt, int64_t nw_max, int t_max, const pm_bucket *buckets,
                         const double *theta0, const double *bg, int64_t B, const int64_t *n_dev, int32_t iters,
                         double beta, double *theta_out, double *J_out, double *llr_out, int32_t *sites_out,
                         void *ws, bool split, hipStream_t st)
{
    uint8_t *w = static_cast<uint8_t *>(ws);
    int64_t *plan = reinterpret_cast<int64_t *>(w);
    int64_t *tbase = reinterpret_cast<int64_t *>(w + plan_bytes(Bt->P));
    uint8_t *tables = w + plan_bytes(Bt->P) + tbase_bytes(Bt->P);
    int shape = tuned_shape(Bt->l, split);
    if (!shape_ok(shape, Bt->l)) shape = 10 + shape % 10;
    hipLaunchKernelGGL(k_em_plan, dim3(1), dim3(1024), 0, st, Bt->inst, Bt->P, buckets, n_dev, B,
                       16 * kWaves * (shape / 10), plan, tbase);
    PM_LAUNCHED();
    EmTabArgs tt{};
    tt.inst = Bt->inst;
    tt.tbase = tbase;
    tt.P = Bt->P;
    tt.l = Bt->l;
    tt.nslots = batch_slots(Bt);
    tt.tables = tables;
    const int rc = launch_em_tables(tt, st);
    if (rc != PM_OK) return rc;
    EmMfmaArgs a{};
    a.split = split;
    a.inst = Bt->inst;
    a.plan = plan;
    a.P = Bt->P;
    a.tables = tables;
    a.tbase = tbase;
    a.theta0 = theta0;
    a.bg = bg;
    a.n_dev = n_dev;
    a.theta_out = theta_out;
    a.J = J_out;
    a.llr = llr_out;
    a.sites = sites_out;
    a.B = B;
    a.site_stride = t_max;
    a.l = Bt->l;
    a.iters = iters;
    a.beta = beta;
    (void)nw_max;
    // every instance wastes at most one partly filled group
    return dispatch_em_mfma(a, st, shape);
}

int em_autotune_mfma(const pm_seqs *S, int32_t l, const double *theta0, const double *bg, int64_t B, int32_t iters,
                     double beta, bool split, double *theta_out, double *J_out, void *ws, size_t ws_bytes,
                     int32_t *choice, hipStream_t st)
{
    EmMfmaArgs a{};
    a.split = split;
    a.packed = S->packed;
    a.offsets = S->offsets;
    a.theta0 = theta0;
    a.bg = bg;
    a.theta_out = theta_out;
    a.J = J_out;
    a.B = B;
    a.nwords = pm_packed_words(S->alphabet, S->n_total);
    a.t = S->t;
    a.site_stride = S->t;
    a.l = l;
    a.iters = iters;
    a.beta = beta;
    const int prc = prepare_tables(a, S, l, ws, ws_bytes, st);
    if (prc != PM_OK) return prc;
    hipEvent_t e0, e1;
    PM_TRY(hipEventCreate(&e0));
    PM_TRY(hipEventCreate(&e1));
    float best_ms = 0.f;
    int best = 0, rc = PM_OK;
    for (const int shape : {11, 12, 14, 21, 22, 24}) {
        if (!shape_ok(shape, l)) continue;
        float ms = 0.f;
        rc = dispatch_em_mfma(a, st, shape);  // warm-up
        if (rc == PM_OK && hipEventRecord(e0, st) != hipSuccess) rc = fail(PM_EDEVICE, "hipEventRecord failed");
        if (rc == PM_OK) rc = dispatch_em_mfma(a, st, shape);
        if (rc == PM_OK && hipEventRecord(e1, st) != hipSuccess) rc = fail(PM_EDEVICE, "hipEventRecord failed");
        if (rc == PM_OK && hipEventSynchronize(e1) != hipSuccess) rc = fail(PM_EDEVICE, "hipEventSynchronize failed");
        if (rc == PM_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = fail(PM_EDEVICE, "hipEventElapsedTime failed");
        if (rc != PM_OK) break;
        if (best == 0 || ms < best_ms) {
            best = shape;
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != PM_OK) return rc;
    g_shape[(l + 3) / 4 - 1][split ? 1 : 0] = best;
    if (choice) *choice = best;
    return PM_OK;
}

int em_tuned_shape(int32_t l, bool split) { return tuned_shape(l, split); }

int em_record_shape(int32_t l, bool split, int32_t shape)
{
    if (!shape_ok(shape, l))
        return fail(PM_EINVAL, "tile shape %d is not one of 11, 12, 14, 21, 22, 24 (G = 2 needs l <= %d)", shape,
                    4 * kMaxMT2);
    g_shape[(l + 3) / 4 - 1][split ? 1 : 0] = shape;
    return PM_OK;
}


}  // namespace pm
