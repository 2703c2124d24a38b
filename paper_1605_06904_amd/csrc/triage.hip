// Learned bucket triage: bucket features, the 87 -> 256 -> 256 -> 1 ReLU
// network (BF16 matrix-core forward for serving, FP32 forward/backward and
// Adam for training), per-instance top-fraction selection and compaction of
// the chosen buckets, and the full-refinement fallback.
//
// The paper refines every enriched bucket (Sec. 5.1); triage is an addition:
// a network trained on (bucket, post-EM score) pairs of the method's own runs
// ranks the buckets of every instance, EM refines only the best-ranked
// fraction, and an instance whose best refined score falls below a threshold
// gets all of its remaining buckets refined after all.
#include <math.h>

#include "pm_common.h"

namespace pm {

constexpr int kIn = 87, kHid = 256, kLmax = 21;
constexpr int64_t oW1 = 0, ob1 = oW1 + (int64_t)kIn * kHid, oW2 = ob1 + kHid, ob2 = oW2 + (int64_t)kHid * kHid,
                  oW3 = ob2 + kHid, ob3 = oW3 + kHid, kParams = ob3 + 1;
static_assert(kParams == PM_TRIAGE_PARAMS, "parameter count");

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float float4v __attribute__((ext_vector_type(4)));

// packed serving weights: W1 and W2 as matrix-core A fragments, then FP32
// b1, b2, w3, b3
constexpr int64_t kW1Frags = 16 * 3 * 64, kW2Frags = 16 * 8 * 64;
constexpr size_t kPackedBytes = (size_t)(kW1Frags + kW2Frags) * 16 + (3 * kHid + 1) * 4;

__device__ __forceinline__ int64_t valid_count(const int64_t *n_dev, int64_t B)
{
    int64_t n = n_dev ? *n_dev : B;
    return n > B ? B : n;
}

// ---------------------------------------------------------------- features
// The PWM block in canonical order: letter counts of a column sorted in
// decreasing order, columns in decreasing lexicographic order of those sorted
// counts (equal keys are equal columns, so the order is unique), as
// frequencies; zeros past column l - 1.
__device__ __forceinline__ void cswap_desc(uint32_t &x, uint32_t &y)
{
    const uint32_t a = x > y ? x : y, b = x > y ? y : x;
    x = a;
    y = b;
}

__device__ __forceinline__ bool lex_greater(const uint32_t (&a)[4], const uint32_t (&b)[4])
{
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (a[j] != b[j]) return a[j] > b[j];
    return false;
}

__global__ void k_tri_features(const uint32_t *__restrict__ prof, int64_t B, const int64_t *n_dev, int l,
                               const double *__restrict__ bg, const float *mu, const float *sd,
                               float *__restrict__ feat)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= valid_count(n_dev, B)) return;
    const uint32_t *P = prof + b * 4 * l;
    float *o = feat + b * kIn;
    const double size = (double)P[0] + P[l] + P[2 * l] + P[3 * l];
    auto put = [&](int i, double v) { o[i] = mu ? (float)((v - (double)mu[i]) / (double)sd[i]) : (float)v; };
    double H = 0, icmax = -INFINITY;
    for (int c = 0; c < 4; ++c)
        if (bg[c] > 0) H -= bg[c] * log2(bg[c]);
    uint32_t sc[kLmax][4];
#pragma unroll
    for (int p = 0; p < kLmax; ++p) {
        uint32_t a[4] = {0u, 0u, 0u, 0u};
        if (p < l) {
            double ic = 0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                a[c] = P[c * l + p];
                const double f = size > 0 ? a[c] / size : 0.0;
                if (f > 0) ic += f * log2(f / bg[c]);
            }
            icmax = ic > icmax ? ic : icmax;
        }
        cswap_desc(a[0], a[1]);
        cswap_desc(a[2], a[3]);
        cswap_desc(a[0], a[2]);
        cswap_desc(a[1], a[3]);
        cswap_desc(a[1], a[2]);
#pragma unroll
        for (int j = 0; j < 4; ++j) sc[p][j] = a[j];
    }
    uint32_t used = 0;
    for (int r = 0; r < kLmax; ++r) {
        uint32_t best[4] = {0u, 0u, 0u, 0u};
        int bi = -1;
        if (r < l) {
#pragma unroll
            for (int p = 0; p < kLmax; ++p)
                if (p < l && !((used >> p) & 1u) && (bi < 0 || lex_greater(sc[p], best))) {
                    bi = p;
#pragma unroll
                    for (int j = 0; j < 4; ++j) best[j] = sc[p][j];
                }
            used |= 1u << bi;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) put(4 * r + j, (r < l && size > 0) ? best[j] / size : 0.0);
    }
    // an empty profile (a bucket cut off by a capacity) gets all-zero raw features
    put(84, size > 0 ? log(size) : 0.0);
    put(85, size > 0 ? H : 0.0);
    put(86, size > 0 ? icmax : 0.0);
}

// ---------------------------------------------------------------- serving
// A fragment of v_mfma_f32_16x16x32_bf16: lane (row r = lane % 16, group
// g = lane / 16) holds K entries 8g .. 8g + 7 of row r.  Layer 1 computes
// Z1^T = W1^T X^T (rows: hidden units, columns: buckets).  Its output tile
// leaves lane (bucket r, group g) with units 4g .. 4g + 3 of the tile, so the
// layer-2 K step ks takes units {32ks + 4g + j, 32ks + 16 + 4g + j : j < 4}
// from two layer-1 tiles straight out of the accumulators; W2's fragments use
// the same order of K.
__device__ __forceinline__ int l2_unit(int ks, int g, int j) { return 32 * ks + (j < 4 ? 4 * g + j : 16 + 4 * g + j - 4); }

__global__ void k_tri_pack(const float *__restrict__ prm, __bf16 *__restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n1 = kW1Frags * 8, n2 = kW2Frags * 8;
    if (e < n1) {
        const int j = e % 8, lane = (e / 8) % 64, ks = (e / 512) % 3, ut = e / 1536;
        const int r = lane % 16, g = lane / 16, in = 32 * ks + 8 * g + j, unit = 16 * ut + r;
        out[e] = (__bf16)(in < kIn ? prm[oW1 + (int64_t)in * kHid + unit] : 0.0f);
    } else if (e < n1 + n2) {
        const int64_t f = e - n1;
        const int j = f % 8, lane = (f / 8) % 64, ks = (f / 512) % 8, ut = f / 4096;
        const int r = lane % 16, g = lane / 16, hin = l2_unit(ks, g, j), hout = 16 * ut + r;
        out[e] = (__bf16)prm[oW2 + (int64_t)hin * kHid + hout];
    } else if (e < n1 + n2 + 3 * kHid + 1) {
        const int q = (int)(e - n1 - n2);
        float *tail = reinterpret_cast<float *>(out + n1 + n2);
        tail[q] = q < kHid ? prm[ob1 + q] : q < 2 * kHid ? prm[ob2 + q - kHid] : q < 3 * kHid ? prm[oW3 + q - 2 * kHid]
                                                                                           : prm[ob3];
    }
}

constexpr int kTriR = 2;  // 16-bucket column tiles per wave

__global__ void __launch_bounds__(256) k_tri_forward(const float *__restrict__ feat, int64_t B, const int64_t *n_dev,
                                                     const bf16x8 *__restrict__ w1f, const bf16x8 *__restrict__ w2f,
                                                     const float *__restrict__ tail, float *__restrict__ score)
{
    const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4, wv = threadIdx.x >> 6;
    const int64_t nvalid = valid_count(n_dev, B);
    const int64_t base = ((int64_t)blockIdx.x * 4 + wv) * 16 * kTriR;
    if (base >= nvalid) return;  // uniform over the wave; no workgroup barriers below
    bf16x8 X[kTriR][3];
#pragma unroll
    for (int c = 0; c < kTriR; ++c) {
        const int64_t b = base + 16 * c + r;
        const bool ok = b < nvalid;
#pragma unroll
        for (int ks = 0; ks < 3; ++ks)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int in = 32 * ks + 8 * g + j;
                X[c][ks][j] = (__bf16)(ok && in < kIn ? feat[b * kIn + in] : 0.0f);
            }
    }
    float4v acc[16][kTriR];
#pragma unroll
    for (int u = 0; u < 16; ++u)
#pragma unroll
        for (int c = 0; c < kTriR; ++c) acc[u][c] = float4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int ks2 = 0; ks2 < 8; ++ks2) {
        bf16x8 H[kTriR];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int ut1 = 2 * ks2 + h;
            float4v z[kTriR];
#pragma unroll
            for (int c = 0; c < kTriR; ++c) z[c] = float4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks1 = 0; ks1 < 3; ++ks1) {
                const bf16x8 A = w1f[(ut1 * 3 + ks1) * 64 + lane];
#pragma unroll
                for (int c = 0; c < kTriR; ++c) z[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, X[c][ks1], z[c], 0, 0, 0);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float bias = tail[16 * ut1 + 4 * g + i];
#pragma unroll
                for (int c = 0; c < kTriR; ++c) H[c][4 * h + i] = (__bf16)fmaxf(z[c][i] + bias, 0.0f);
            }
        }
#pragma unroll
        for (int ut2 = 0; ut2 < 16; ++ut2) {
            const bf16x8 A = w2f[(ut2 * 8 + ks2) * 64 + lane];
#pragma unroll
            for (int c = 0; c < kTriR; ++c) acc[ut2][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, H[c], acc[ut2][c], 0, 0, 0);
        }
    }
    float y[kTriR];
#pragma unroll
    for (int c = 0; c < kTriR; ++c) y[c] = 0.f;
#pragma unroll
    for (int ut2 = 0; ut2 < 16; ++ut2)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int u = 16 * ut2 + 4 * g + i;
            const float b2 = tail[kHid + u], w3 = tail[2 * kHid + u];
#pragma unroll
            for (int c = 0; c < kTriR; ++c) y[c] += fmaxf(acc[ut2][c][i] + b2, 0.0f) * w3;
        }
#pragma unroll
    for (int c = 0; c < kTriR; ++c) {
        y[c] += __shfl_xor(y[c], 16);
        y[c] += __shfl_xor(y[c], 32);
        const int64_t b = base + 16 * c + r;
        if (g == 0 && b < nvalid) score[b] = y[c] + tail[3 * kHid];
    }
}

// ---------------------------------------------------------------- training (FP32)
// C[M x N] = op(A) op(B) (+ bias[N]) (ReLU) (* [mask > 0]); op(A) = A^T when
// TA (A stored K x M), op(B) = B^T when TB (B stored N x K).  64 x 64 tiles,
// a 4 x 4 block per thread, K in steps of 16 in a fixed order (deterministic).
template <bool TA, bool TB>
__global__ void __launch_bounds__(256) k_gemm(const float *__restrict__ A, const float *__restrict__ Bm,
                                              float *__restrict__ Cm, int M, int N, int K, int lda, int ldb, int ldc,
                                              const float *bias, int relu, const float *mask)
{
    __shared__ float As[16][68], Bs[16][68];
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = tid + 256 * e;
            const int mm = TA ? idx % 64 : idx / 16, kk = TA ? idx / 64 : idx % 16;
            const int gm = m0 + mm, gk = k0 + kk;
            As[kk][mm] = (gm < M && gk < K) ? (TA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk]) : 0.f;
            const int nn = TB ? idx / 16 : idx % 64, kb = TB ? idx % 16 : idx / 64;
            const int gn = n0 + nn, gkb = k0 + kb;
            Bs[kb][nn] = (gn < N && gkb < K) ? (TB ? Bm[(int64_t)gn * ldb + gkb] : Bm[(int64_t)gkb * ldb + gn]) : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a[i] = As[kk][ty * 4 + i];
                b[i] = Bs[kk][tx * 4 + i];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int gm = m0 + ty * 4 + i, gn = n0 + tx * 4 + j;
            if (gm >= M || gn >= N) continue;
            float v = acc[i][j] + (bias ? bias[gn] : 0.f);
            if (relu) v = fmaxf(v, 0.f);
            if (mask && !(mask[(int64_t)gm * ldc + gn] > 0.f)) v = 0.f;
            Cm[(int64_t)gm * ldc + gn] = v;
        }
}

// out[c] = sum_n w[n] M[n][c] (w = 1 when NULL), rows in order
__global__ void k_colsum(const float *__restrict__ Mx, int N, int C, int ld, const float *w, float *__restrict__ out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    float s = 0.f;
    for (int n = 0; n < N; ++n) s = fmaf(w ? w[n] : 1.f, Mx[(int64_t)n * ld + c], s);
    out[c] = s;
}

__global__ void k_tri_dy(const float *__restrict__ y, const float *__restrict__ target, int N, float *__restrict__ dy,
                         float *__restrict__ sq)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const float e = y[n] - target[n];
    dy[n] = 2.f * e / (float)N;
    sq[n] = e * e / (float)N;
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       int64_t n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------- selection
// Order-preserving map of a float score to an unsigned key (larger score ->
// larger key); NaN maps below everything.
__device__ __forceinline__ uint32_t score_key(float s)
{
    if (s != s) return 0u;
    const uint32_t u = __float_as_uint(s);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

struct SelView {
    uint32_t *hist;    // [P][256]
    uint32_t *prefix;  // [P] key bits fixed so far
    uint32_t *need;    // [P] rank still to find inside the prefix
    int64_t *range;    // [P][2] bucket range of each instance
    int32_t *mode;     // [P] 0: top fraction, 1: every bucket not taken before, 2: none
    int64_t *blk;      // [nblk + 1] compaction block offsets
};

static SelView sel_view(void *ws, int P, int64_t nblk)
{
    char *p = static_cast<char *>(ws);
    SelView v;
    v.range = reinterpret_cast<int64_t *>(p);
    v.blk = v.range + 2 * (int64_t)P;
    v.hist = reinterpret_cast<uint32_t *>(v.blk + nblk + 1);
    v.prefix = v.hist + 256 * (int64_t)P;
    v.need = v.prefix + P;
    v.mode = reinterpret_cast<int32_t *>(v.need + P);
    return v;
}

constexpr int kSelBlock = 1024;

// bucket range of every instance (buckets ascend by item); rank to find
__global__ void k_tsel_init(const pm_inst *inst, int P, const pm_bucket *buckets, const int64_t *n_dev, int64_t B,
                            double frac, SelView v)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int64_t nvalid = valid_count(n_dev, B);
    int64_t r[2] = {0, nvalid};
    if (inst) {
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
    }
    v.range[2 * p] = r[0];
    v.range[2 * p + 1] = r[1];
    const int64_t n = r[1] - r[0];
    int64_t c = (int64_t)ceil(frac * (double)n);
    if (c < 1) c = 1;
    if (c > n) c = n;
    v.need[p] = (uint32_t)c;
    v.prefix[p] = 0;
    for (int i = 0; i < 256; ++i) v.hist[256 * (int64_t)p + i] = 0;
}

__device__ __forceinline__ int inst_of_bucket(const int32_t *item_inst, const pm_bucket *buckets, int64_t b)
{
    return item_inst ? item_inst[buckets[b].trial] : 0;
}

// histogram of digit `pass` (8 bits, most significant first) of the keys
// that match the instance's prefix so far
__global__ void __launch_bounds__(256) k_tsel_hist(const float *score, const int32_t *item_inst,
                                                   const pm_bucket *buckets, const int64_t *n_dev, int64_t B, int pass,
                                                   SelView v)
{
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= valid_count(n_dev, B)) return;
    const int p = inst_of_bucket(item_inst, buckets, b);
    const uint32_t key = score_key(score[b]);
    const int sh = 24 - 8 * pass;
    const uint32_t hi_mask = pass == 0 ? 0u : (0xffffffffu << (sh + 8));
    if ((key & hi_mask) != (v.prefix[p] & hi_mask)) return;
    atomicAdd(v.hist + 256 * (int64_t)p + ((key >> sh) & 255u), 1u);
}

// per instance: the digit holding the need-th largest key, then clear
__global__ void k_tsel_pick(int P, int pass, SelView v)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    uint32_t *h = v.hist + 256 * (int64_t)p;
    const int sh = 24 - 8 * pass;
    uint32_t need = v.need[p];
    if (need == 0) return;  // empty instance
    int d = 255;
    for (; d > 0; --d) {
        if (h[d] >= need) break;
        need -= h[d];
    }
    v.prefix[p] |= (uint32_t)d << sh;
    v.need[p] = need;
    for (int i = 0; i < 256; ++i) h[i] = 0;
}

// keep flag of a bucket under its instance's mode
__device__ __forceinline__ bool tsel_keep(const float *score, const int32_t *item_inst, const pm_bucket *buckets,
                                          const uint8_t *taken, const SelView &v, int64_t b)
{
    const int p = inst_of_bucket(item_inst, buckets, b);
    const int md = v.mode[p];
    if (md == 0) return v.need[p] > 0 && score_key(score[b]) >= v.prefix[p];
    if (md == 1) return !(taken && taken[b]);
    return false;
}

__global__ void __launch_bounds__(256) k_tsel_count(const float *score, const int32_t *item_inst,
                                                    const pm_bucket *buckets, const int64_t *n_dev, int64_t B,
                                                    const uint8_t *taken, SelView v)
{
    const int64_t nvalid = valid_count(n_dev, B);
    const int64_t b0 = (int64_t)blockIdx.x * kSelBlock;
    uint32_t c = 0;
    for (int64_t b = b0 + threadIdx.x; b < b0 + kSelBlock && b < nvalid; b += 256)
        c += tsel_keep(score, item_inst, buckets, taken, v, b) ? 1u : 0u;
    c = wave_sum(c);
    __shared__ uint32_t red[4];
    if (lane_id() == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) v.blk[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void __launch_bounds__(1024) k_tsel_scan(int64_t nblk, SelView v, int64_t *n_sel)
{
    __shared__ int64_t s[1024];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nblk; base += 1024) {
        const int64_t j = base + threadIdx.x;
        const int64_t x = j < nblk ? v.blk[j] : 0;
        s[threadIdx.x] = x;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int64_t u = (int)threadIdx.x >= o ? s[threadIdx.x - o] : 0;
            __syncthreads();
            s[threadIdx.x] += u;
            __syncthreads();
        }
        if (j < nblk) v.blk[j] = carry + s[threadIdx.x] - x;
        __syncthreads();
        if (threadIdx.x == 1023) carry += s[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        v.blk[nblk] = carry;
        *n_sel = carry;
    }
}

// stable compaction: block offsets from the scan, order inside a block by a
// wave-by-wave prefix of the keep flags
__global__ void __launch_bounds__(256) k_tsel_emit(const float *score, const int32_t *item_inst,
                                                   const pm_bucket *buckets, const int64_t *n_dev, int64_t B,
                                                   uint8_t *taken, SelView v, const double *theta0, int AL,
                                                   pm_bucket *sel_buckets, double *sel_theta0, int64_t *sel_index)
{
    const int64_t nvalid = valid_count(n_dev, B);
    const int64_t b0 = (int64_t)blockIdx.x * kSelBlock;
    __shared__ uint32_t wtot[4];
    __shared__ int64_t run;
    if (threadIdx.x == 0) run = v.blk[blockIdx.x];
    __syncthreads();
    const int wv = threadIdx.x >> 6;
    for (int64_t c0 = b0; c0 < b0 + kSelBlock; c0 += 256) {
        const int64_t b = c0 + threadIdx.x;
        const bool ok = b < nvalid && b < b0 + kSelBlock;
        const bool keep = ok && tsel_keep(score, item_inst, buckets, taken, v, b);
        const uint64_t bal = __ballot(keep);
        if (lane_id() == 0) wtot[wv] = __popcll(bal);
        __syncthreads();
        int64_t pos = run;
        for (int w = 0; w < wv; ++w) pos += wtot[w];
        pos += __popcll(bal & lanemask_lt());
        if (keep) {
            sel_buckets[pos] = buckets[b];
            if (sel_index) sel_index[pos] = b;
            for (int i = 0; i < AL; ++i) sel_theta0[pos * AL + i] = theta0[b * AL + i];
            if (taken) taken[b] = 1;
        }
        __syncthreads();
        if (threadIdx.x == 0) run += wtot[0] + wtot[1] + wtot[2] + wtot[3];
        __syncthreads();
    }
}

__global__ void k_fill_u8(uint8_t *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void k_tsel_mode(int P, SelView v, int32_t mode)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < P) v.mode[p] = mode;
}

// fallback decision, one workgroup per instance: the z-score of the triaged
// winner's J among the J of every bucket the instance refined (list 1); an
// instance whose winner does not stand out by the threshold (or that refined
// nothing) gets every other bucket refined
__device__ __forceinline__ double block_sum_f64(double v, double *red)
{
    v = wave_sum(v);
    __syncthreads();
    if (lane_id() == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

__global__ void __launch_bounds__(256) k_tsel_fallback(int P, const pm_inst *inst, const pm_bucket *sel1,
                                                       const int64_t *n_sel1, const int64_t *best, const double *J,
                                                       int iters, double threshold, SelView v, int32_t *fell_back,
                                                       double *z_out)
{
    __shared__ double red[4];
    const int p = blockIdx.x;
    const int64_t n1 = *n_sel1;
    int64_t r[2] = {0, n1};
    if (inst) {
        for (int side = 0; side < 2; ++side) {
            const int64_t item = (int64_t)inst[p].first_item + (side ? inst[p].m : 0);
            int64_t lo = 0, hi = n1;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if ((int64_t)sel1[mid].trial < item) lo = mid + 1;
                else hi = mid;
            }
            r[side] = lo;
        }
    }
    const int64_t n = r[1] - r[0];
    double s = 0;
    for (int64_t b = r[0] + threadIdx.x; b < r[1]; b += 256) s += J[b * (iters + 1) + iters];
    const double mean = n > 0 ? block_sum_f64(s, red) / (double)n : 0.0;
    double q = 0;
    for (int64_t b = r[0] + threadIdx.x; b < r[1]; b += 256) {
        const double d = J[b * (iters + 1) + iters] - mean;
        q += d * d;
    }
    const double sd = n > 0 ? sqrt(block_sum_f64(q, red) / (double)n) : 0.0;
    if (threadIdx.x != 0) return;
    const int64_t bb = best[p];
    double z = -INFINITY;
    if (bb >= 0) z = sd > 0 ? (J[bb * (iters + 1) + iters] - mean) / sd : 0.0;
    const bool low = !(z >= threshold);
    const bool any = v.range[2 * p + 1] > v.range[2 * p];
    v.mode[p] = (low && any) ? 1 : 2;
    if (fell_back) fell_back[p] = (low && any) ? 1 : 0;
    if (z_out) z_out[p] = z;
}

// per instance: the better of the triaged winner and the fallback winner, as
// an index into the original bucket list, with its consensus
__global__ void k_tsel_merge(int P, int A, int l, int iters, const int64_t *best1, const int64_t *idx1, const double *J1,
                             const double *th1, const int64_t *best2, const int64_t *idx2, const double *J2,
                             const double *th2, int64_t *best_out, char *cons)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int64_t a = best1[p], b = best2 ? best2[p] : -1;
    const double ja = a >= 0 ? J1[a * (iters + 1) + iters] : -INFINITY;
    const double jb = b >= 0 ? J2[b * (iters + 1) + iters] : -INFINITY;
    // larger J wins; on a tie the lower original bucket index
    bool use_b = false;
    if (b >= 0 && (a < 0 || jb > ja || (jb == ja && idx2[b] < idx1[a]))) use_b = true;
    const int64_t w = use_b ? b : a;
    best_out[p] = w < 0 ? -1 : (use_b ? idx2[w] : idx1[w]);
    if (!cons) return;
    const double *th = use_b ? th2 : th1;
    const char *letters = A == 4 ? "ACTG" : "ARNDCQEGHILKMFPSTWYV";
    char *o = cons + (int64_t)p * (l + 1);
    for (int q = 0; q < l; ++q) {
        char ch = 0;
        if (w >= 0) {
            int bc = 0;
            for (int c = 1; c < A; ++c)
                if (th[(w * A + c) * l + q] > th[(w * A + bc) * l + q]) bc = c;
            ch = letters[bc];
        }
        o[q] = ch;
    }
    o[l] = 0;
}

}  // namespace pm

using namespace pm;

extern "C" size_t pm_triage_packed_bytes(void) { return kPackedBytes; }

extern "C" int triage_pack(const float *params, void *packed, void *stream)
{
    clear_error();
    if (!params || !packed) return fail(PM_EINVAL, "NULL buffer");
    const int64_t n = (kW1Frags + kW2Frags) * 8 + 3 * kHid + 1;
    hipLaunchKernelGGL(k_tri_pack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, as_stream(stream), params,
                       static_cast<__bf16 *>(packed));
    PM_LAUNCHED();
    return PM_OK;
}

extern "C" int triage_features(int32_t l, const uint32_t *profile, int64_t B, const int64_t *n_dev, const double *bg,
                               const float *mu, const float *sd, float *feat, void *stream)
{
    clear_error();
    if (l < 1 || l > kLmax) return fail(PM_EINVAL, "triage features need 1 <= l <= %d", kLmax);
    if (B < 0) return fail(PM_EINVAL, "B must be >= 0");
    if (B == 0) return PM_OK;
    if (!profile || !bg || !feat || (!mu) != (!sd)) return fail(PM_EINVAL, "NULL buffer");
    hipLaunchKernelGGL(k_tri_features, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, as_stream(stream), profile, B,
                       n_dev, l, bg, mu, sd, feat);
    PM_LAUNCHED();
    return PM_OK;
}

extern "C" int triage_forward(const void *packed, const float *feat, int64_t B, const int64_t *n_dev, float *score,
                              void *stream)
{
    clear_error();
    if (B < 0) return fail(PM_EINVAL, "B must be >= 0");
    if (B == 0) return PM_OK;
    if (!packed || !feat || !score) return fail(PM_EINVAL, "NULL buffer");
    const bf16x8 *w1f = static_cast<const bf16x8 *>(packed);
    const bf16x8 *w2f = w1f + kW1Frags;
    const float *tail = reinterpret_cast<const float *>(w2f + kW2Frags);
    const int64_t per_wg = 4 * 16 * kTriR;
    hipLaunchKernelGGL(k_tri_forward, dim3((unsigned)((B + per_wg - 1) / per_wg)), dim3(256), 0, as_stream(stream),
                       feat, B, n_dev, w1f, w2f, tail, score);
    PM_LAUNCHED();
    return PM_OK;
}

extern "C" size_t pm_triage_workspace(int32_t N)
{
    if (N < 1) return 0;
    return ((size_t)4 * N * kHid + 3 * (size_t)N + kParams + 1) * sizeof(float) + 256;
}

template <bool TA, bool TB>
static void gemm(const float *A, const float *B, float *C, int M, int N, int K, int lda, int ldb, int ldc,
                 const float *bias, int relu, const float *mask, hipStream_t st)
{
    dim3 grid((N + 63) / 64, (M + 63) / 64);
    hipLaunchKernelGGL((k_gemm<TA, TB>), grid, dim3(256), 0, st, A, B, C, M, N, K, lda, ldb, ldc, bias, relu, mask);
}

extern "C" int triage_train_step(float *params, float *adam_m, float *adam_v, int32_t step, const float *X,
                                 const float *target, int32_t N, float lr, float *loss_out, float *grads_out,
                                 void *ws, size_t ws_bytes, void *stream)
{
    clear_error();
    if (N < 1) return fail(PM_EINVAL, "N must be >= 1");
    if (!params || !X || !target || !ws) return fail(PM_EINVAL, "NULL buffer");
    if (ws_bytes < pm_triage_workspace(N)) return fail(PM_EINVAL, "workspace too small");
    if (lr > 0 && (!adam_m || !adam_v || step < 1)) return fail(PM_EINVAL, "Adam needs its moments and step >= 1");
    hipStream_t st = as_stream(stream);
    float *H1 = static_cast<float *>(ws), *H2 = H1 + (int64_t)N * kHid, *dZ2 = H2 + (int64_t)N * kHid;
    float *dZ1 = dZ2 + (int64_t)N * kHid, *y = dZ1 + (int64_t)N * kHid, *dy = y + N, *sq = dy + N;
    float *grads = sq + N, *lossb = grads + kParams;
    float *G = grads_out ? grads_out : grads;
    const float *W1 = params + oW1, *b1 = params + ob1, *W2 = params + oW2, *b2 = params + ob2;
    const float *W3 = params + oW3, *b3 = params + ob3;
    // forward
    gemm<false, false>(X, W1, H1, N, kHid, kIn, kIn, kHid, kHid, b1, 1, nullptr, st);
    gemm<false, false>(H1, W2, H2, N, kHid, kHid, kHid, kHid, kHid, b2, 1, nullptr, st);
    gemm<false, false>(H2, W3, y, N, 1, kHid, kHid, 1, 1, b3, 0, nullptr, st);
    hipLaunchKernelGGL(k_tri_dy, dim3((N + 255) / 256), dim3(256), 0, st, y, target, N, dy, sq);
    hipLaunchKernelGGL(k_colsum, dim3(1), dim3(64), 0, st, sq, N, 1, 1, nullptr, loss_out ? loss_out : lossb);
    // backward
    gemm<true, false>(H2, dy, G + oW3, kHid, 1, N, kHid, 1, 1, nullptr, 0, nullptr, st);
    hipLaunchKernelGGL(k_colsum, dim3(1), dim3(64), 0, st, dy, N, 1, 1, nullptr, G + ob3);
    gemm<false, false>(dy, W3, dZ2, N, kHid, 1, 1, kHid, kHid, nullptr, 0, H2, st);
    gemm<true, false>(H1, dZ2, G + oW2, kHid, kHid, N, kHid, kHid, kHid, nullptr, 0, nullptr, st);
    hipLaunchKernelGGL(k_colsum, dim3(1), dim3(256), 0, st, dZ2, N, kHid, kHid, nullptr, G + ob2);
    gemm<false, true>(dZ2, W2, dZ1, N, kHid, kHid, kHid, kHid, kHid, nullptr, 0, H1, st);
    gemm<true, false>(X, dZ1, G + oW1, kIn, kHid, N, kIn, kHid, kHid, nullptr, 0, nullptr, st);
    hipLaunchKernelGGL(k_colsum, dim3(1), dim3(256), 0, st, dZ1, N, kHid, kHid, nullptr, G + ob1);
    if (lr > 0) {
        const float b1m = 0.9f, b2m = 0.999f;
        const float c1 = 1.f - powf(b1m, (float)step), c2 = 1.f - powf(b2m, (float)step);
        hipLaunchKernelGGL(k_adam, dim3((unsigned)((kParams + 255) / 256)), dim3(256), 0, st, params, G, adam_m, adam_v,
                           kParams, lr, b1m, b2m, 1e-8f, c1, c2);
    }
    PM_LAUNCHED();
    return PM_OK;
}

extern "C" size_t pm_triage_select_workspace(int32_t P, int64_t B)
{
    if (P < 1 || B < 0) return 0;
    const int64_t nblk = (B + kSelBlock - 1) / kSelBlock;
    return (size_t)(2 * (int64_t)P + nblk + 1) * 8 + (size_t)P * (256 + 3) * 4 + 256;
}

static int tsel_args(const pm_batch *Bt, int64_t B, const pm_bucket *buckets, const float *score,
                     const double *theta0, int32_t A, int32_t l, pm_bucket *sel_buckets, double *sel_theta0,
                     int64_t *n_sel, void *ws, size_t ws_bytes, int *P)
{
    if (Bt) {
        int rc = check_batch(Bt, nullptr);
        if (rc) return rc;
        if (Bt->alphabet != A || Bt->l != l) return fail(PM_EINVAL, "alphabet/l differ from the batch");
    }
    *P = Bt ? Bt->P : 1;
    if (A != 4 && A != 20) return fail(PM_EINVAL, "alphabet must be 4 or 20");
    if (l < 1 || l > 32 || B < 0) return fail(PM_EINVAL, "bad sizes");
    if (B > 0 && (!buckets || !score || !theta0 || !sel_buckets || !sel_theta0 || !n_sel))
        return fail(PM_EINVAL, "NULL buffer");
    if (!ws || ws_bytes < pm_triage_select_workspace(*P, B)) return fail(PM_EINVAL, "workspace too small");
    return PM_OK;
}

static void tsel_compact(const float *score, const int32_t *item_inst, const pm_bucket *buckets,
                         const int64_t *n_dev, int64_t B, uint8_t *taken, const SelView &v, int64_t nblk,
                         const double *theta0, int AL, pm_bucket *sel_buckets, double *sel_theta0, int64_t *sel_index,
                         int64_t *n_sel, hipStream_t st)
{
    hipLaunchKernelGGL(k_tsel_count, dim3((unsigned)nblk), dim3(256), 0, st, score, item_inst, buckets, n_dev, B, taken,
                       v);
    hipLaunchKernelGGL(k_tsel_scan, dim3(1), dim3(1024), 0, st, nblk, v, n_sel);
    hipLaunchKernelGGL(k_tsel_emit, dim3((unsigned)nblk), dim3(256), 0, st, score, item_inst, buckets, n_dev, B, taken,
                       v, theta0, AL, sel_buckets, sel_theta0, sel_index);
}

extern "C" int triage_select(const pm_batch *Bt, const pm_bucket *buckets, const float *score, int64_t B,
                             const int64_t *n_dev, double frac, const double *theta0, int32_t A, int32_t l,
                             uint8_t *taken, pm_bucket *sel_buckets, double *sel_theta0, int64_t *sel_index,
                             int64_t *n_sel, void *ws, size_t ws_bytes, void *stream)
{
    clear_error();
    int P = 1;
    int rc = tsel_args(Bt, B, buckets, score, theta0, A, l, sel_buckets, sel_theta0, n_sel, ws, ws_bytes, &P);
    if (rc) return rc;
    if (!(frac > 0 && frac <= 1)) return fail(PM_EINVAL, "frac must be in (0, 1]");
    if (B == 0) return PM_OK;
    hipStream_t st = as_stream(stream);
    const int64_t nblk = (B + kSelBlock - 1) / kSelBlock;
    const SelView v = sel_view(ws, P, nblk);
    const pm_inst *inst = Bt ? Bt->inst : nullptr;
    const int32_t *item_inst = Bt ? Bt->item_inst : nullptr;
    const unsigned pg = (unsigned)((P + 255) / 256);
    if (taken) hipLaunchKernelGGL(k_fill_u8, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, st, taken, B);
    hipLaunchKernelGGL(k_tsel_init, dim3(pg), dim3(256), 0, st, inst, P, buckets, n_dev, B, frac, v);
    hipLaunchKernelGGL(k_tsel_mode, dim3(pg), dim3(256), 0, st, P, v, 0);
    for (int pass = 0; pass < 4; ++pass) {
        hipLaunchKernelGGL(k_tsel_hist, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, st, score, item_inst, buckets,
                           n_dev, B, pass, v);
        hipLaunchKernelGGL(k_tsel_pick, dim3(pg), dim3(256), 0, st, P, pass, v);
    }
    tsel_compact(score, item_inst, buckets, n_dev, B, taken, v, nblk, theta0, A * l, sel_buckets, sel_theta0, sel_index,
                 n_sel, st);
    PM_LAUNCHED();
    return PM_OK;
}

extern "C" int triage_fallback_select(const pm_batch *Bt, const pm_bucket *buckets, int64_t B, const int64_t *n_dev,
                                      const pm_bucket *sel1, const int64_t *n_sel1, const int64_t *best,
                                      const double *J, int32_t iters, double threshold, const double *theta0,
                                      int32_t A, int32_t l, uint8_t *taken, pm_bucket *sel_buckets,
                                      double *sel_theta0, int64_t *sel_index, int64_t *n_sel, int32_t *fell_back,
                                      double *z_out, void *ws, size_t ws_bytes, void *stream)
{
    clear_error();
    int P = 1;
    const float dummy = 0.f;
    int rc = tsel_args(Bt, B, buckets, &dummy, theta0, A, l, sel_buckets, sel_theta0, n_sel, ws, ws_bytes, &P);
    if (rc) return rc;
    if (!best || !J || !taken || !sel1 || !n_sel1 || iters < 0) return fail(PM_EINVAL, "NULL buffer");
    if (B == 0) return PM_OK;
    hipStream_t st = as_stream(stream);
    const int64_t nblk = (B + kSelBlock - 1) / kSelBlock;
    const SelView v = sel_view(ws, P, nblk);
    const pm_inst *inst = Bt ? Bt->inst : nullptr;
    // ranges are those of the preceding triage_select on the same workspace
    hipLaunchKernelGGL(k_tsel_fallback, dim3((unsigned)P), dim3(256), 0, st, P, inst, sel1, n_sel1, best, J, iters,
                       threshold, v, fell_back, z_out);
    tsel_compact(nullptr, Bt ? Bt->item_inst : nullptr, buckets, n_dev, B, taken, v, nblk, theta0, A * l, sel_buckets,
                 sel_theta0, sel_index, n_sel, st);
    PM_LAUNCHED();
    return PM_OK;
}

extern "C" int triage_merge_best(int32_t P, int32_t alphabet, int32_t l, int32_t iters, const int64_t *best1,
                                 const int64_t *index1, const double *J1, const double *theta1, const int64_t *best2,
                                 const int64_t *index2, const double *J2, const double *theta2, int64_t *best_out,
                                 char *consensus_out, void *stream)
{
    clear_error();
    if (P < 1 || (alphabet != 4 && alphabet != 20) || l < 1 || l > 32 || iters < 0) return fail(PM_EINVAL, "bad sizes");
    if (!best1 || !index1 || !J1 || !theta1 || !best_out) return fail(PM_EINVAL, "NULL buffer");
    if (best2 && (!index2 || !J2 || !theta2)) return fail(PM_EINVAL, "NULL buffer");
    hipLaunchKernelGGL(k_tsel_merge, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, as_stream(stream), P, alphabet,
                       l, iters, best1, index1, J1, theta1, best2, index2, J2, theta2, best_out, consensus_out);
    PM_LAUNCHED();
    return PM_OK;
}
