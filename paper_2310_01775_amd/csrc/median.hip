// Bandwidth of the SVGD kernel by the median heuristic (Appendix D-B): the
// lower median m2 of the P = N(N-1)/2 squared distances D_ij (i < j, FP32 by
// direct differences in coordinate order), h = max(m2 / ln N, 1e-12).
//
// Exact path (interval select).  Non-negative floats order like their bit
// patterns, so the median is the rank-k bit pattern, k = ceil(P/2).
//   1. A fixed sample of kMedSample pairs is measured (the same squared
//      distances, summed in a fixed order of their own, so within rounding of
//      the passes' values) and its order statistics at ranks
//      S(1/2 -+ 2/sqrt S) give a bracket [lo, hi] that holds rank k unless the
//      sample is off by four standard deviations (about once in 16 000
//      selects; a rank outside it sends the passes back over every pair, step
//      3, so the result stays exact).  A wider bracket makes every pass 0
//      stage and every candidate pass read more candidates.  When all pairs fit in the
//      sample, it is the population and its median is final.  The sample sits
//      in LDS for the select.
//   2. Pass 0 over every pair counts the pairs below lo and above hi and
//      copies the in-bracket bit patterns into a candidate buffer.
//   3. Each later pass histograms the current interval [lo, hi] into 2048
//      linear bins and a select step narrows the interval to the bin holding
//      rank k (with k's rank inside it).  The passes read the candidates when
//      they cover the interval, else every pair again (rank k outside the
//      bracket, or the buffer overflowed).  Widths are below 2^32 and each
//      pass divides them by 2048, so three passes end at a single value.
// Every count is an integer and every comparison exact, so the result is the
// exact order statistic, independent of scheduling.
//
// Problems with at most 2^20 pairs finish after pass 0 in one workgroup of
// 1024 that reads the candidates once into registers and histograms them there
// (or, rarely, runs the passes over every pair), so their select takes four
// kernels.
//
// An all-pairs work item is (ROWS-row block, 64-column chunk) in a workgroup of
// 256: each thread keeps its row's coordinates in registers and reads the
// staged columns as LDS broadcasts, four columns at a time.  Counts go to a
// per-item array (no shared counters); a wave gathers its in-bracket values in
// LDS and appends them to one of kCandSegs buffer segments with one atomic per
// flush, so the segments hold candidates only.
//
// Sampled path: the bandwidth from the sample's own lower median.
#include <math.h>

#include <type_traits>

#include "bf16_operands.h"
#include "common.h"
#include "internal.h"

namespace stamp {

typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f4v;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8v;

namespace {

constexpr uint32_t kModeDone = 0, kModePass0 = 1, kModeCand = 2, kModeAll = 3;
constexpr float kBracketSigmas = 4.0f;
constexpr uint32_t kWaveBuf = 512;        // candidates a wave stages in LDS between flushes
constexpr int kGramGroup = 2;             // column chunks of one Gram-form item
constexpr uint32_t kSentinel = 0xffffffffu;  // above every candidate interval
constexpr int kSelThreads = 1024;         // threads of the sample select

__device__ __forceinline__ uint32_t mix32(uint32_t x) {  // MurmurHash3 finaliser
    x ^= x >> 16;
    x *= 0x85ebca6bu;
    x ^= x >> 13;
    x *= 0xc2b2ae35u;
    x ^= x >> 16;
    return x;
}

__host__ __device__ __forceinline__ uint64_t pair_count(int N) { return (uint64_t)N * (uint64_t)(N - 1) / 2; }

// Bin shift so that an interval of `width` bit patterns fits 2048 bins.
// The smallest s with ceil(width / 2^s) <= 2048, i.e. bitlen(width - 1) - 11.
__device__ __forceinline__ uint32_t shift_for(uint64_t width) {
    const uint64_t m = width - 1;
    const int bl = m ? 64 - __clzll((long long)m) : 0;
    return bl > 11 ? (uint32_t)(bl - 11) : 0u;
}

// One problem's select workspace.
struct MedView {
    int N, d;
    float fixed_h;
    int rows, rb, cc;    // all-pairs items: rows each, row blocks, column chunks
    uint32_t cap;        // candidate slots (kCandSegs segments)
    float* smp;
    SelState* sel;
    uint32_t* hist;
    uint32_t* cand;
    uint32_t* cnt;       // [rb * cc][2]: pairs under, over the bracket
    const float* xr;     // Gram form: centred rows in MFMA operand order (4 ks floats each)
    const float* nrm;    // and their squared norms (FP32 matrix-core operands)
    const __bf16* xs3;   // split form (d <= 31): the same rows as three BF16 parts, [npad][3][32]
};

__device__ __forceinline__ MedView med_view(int N, int d, float fixed_h, const SvgdLayout& L, char* b) {
    MedView v;
    v.N = N;
    v.d = d;
    v.fixed_h = fixed_h;
    v.rows = L.med_rows;
    v.rb = L.med_rb;
    v.cc = L.med_cc;
    v.cap = L.cand_cap;
    v.smp = reinterpret_cast<float*>(b + L.smp_off);
    v.sel = reinterpret_cast<SelState*>(b + L.sel_off);
    v.hist = reinterpret_cast<uint32_t*>(b + L.hist_off);
    v.cand = reinterpret_cast<uint32_t*>(b + L.cand_off);
    v.cnt = reinterpret_cast<uint32_t*>(b + L.cnt_off);
    v.xr = reinterpret_cast<const float*>(b + L.x32_off);
    v.nrm = reinterpret_cast<const float*>(b + L.n32_off);
    v.xs3 = reinterpret_cast<const __bf16*>(b + L.xs3_off);
    return v;
}

// Sample slot t: pair t of the row-major enumeration of i < j when all pairs
// fit (N <= 128), else a hashed pair i != j (oriented i < j, as in the
// all-pairs passes); false beyond the sample.
__device__ bool sample_pair(int N, int t, int& i, int& j) {
    const uint64_t P = pair_count(N);
    const bool all = P <= (uint64_t)kMedSample;
    if (N < 2 || (all && (uint64_t)t >= P)) return false;
    if (all) {
        int r = t;
        i = 0;
        while (r >= N - 1 - i) {
            r -= N - 1 - i;
            ++i;
        }
        j = i + 1 + r;
    } else {
        i = (int)(mix32(2u * (uint32_t)t + 1u) % (uint32_t)N);
        j = (int)(mix32((2u * (uint32_t)t + 2u) ^ 0x9e3779b9u) % (uint32_t)(N - 1));
        if (j >= i) ++j;
        if (j < i) {
            const int x = i;
            i = j;
            j = x;
        }
    }
    return true;
}

// Slot t's squared distance (+inf beyond the sample), by the four lanes q of
// a DPP quad: lane q adds coordinates q, q + 4, q + 8, ... in order (eight
// gathers of each particle in flight, indices clamped so no load is
// predicated) and the quad adds its four sums as (s0 + s1) + (s2 + s3).  The
// random gathers are what a sample slot costs; four lanes per slot put four
// times the waves on them.  Every lane of the quad must call this.
__device__ float sample_dist4(int N, int d, int t, int q, const float* __restrict__ theta) {
    int i = 0, j = 0;
    const bool ok = sample_pair(N, t, i, j);
    float acc = 0.0f;
    if (ok) {
        const float* ti = theta + i;
        const float* tj = theta + j;
        for (int l0 = 0; l0 < d; l0 += 32) {
            float a[8], b[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t o = (int64_t)min(l0 + q + 4 * u, d - 1) * N;
                a[u] = ti[o];
                b[u] = tj[o];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (l0 + q + 4 * u < d) {
                    const float df = a[u] - b[u];
                    acc = fmaf(df, df, acc);
                }
        }
    }
    const float s = quad_sum(acc);
    return ok ? s : __int_as_float(0x7f800000);
}

__device__ __forceinline__ void set_bandwidth(SelState* sel, int N, uint32_t m2_bits, float* h_out) {
    const float m2 = __uint_as_float(m2_bits);
    const float h = fmaxf(m2 / logf((float)N), 1e-12f);
    sel->m2 = m2;
    sel->h = h;
    sel->mode = kModeDone;
    if (h_out) *h_out = h;
}

// ---- select inside one workgroup of NT threads -----------------------------------
// Sum over the workgroup (every thread gets the total); wt: NT/64 words of LDS.
template <int NT>
__device__ __forceinline__ uint32_t wg_sum(uint32_t c, uint32_t* wt) {
    static_assert(NT % 256 == 0, "wave totals are read four at a time");
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0) wt[threadIdx.x >> 6] = c;
    __syncthreads();
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; w += 4) {
        const uint4 v = *reinterpret_cast<const uint4*>(&wt[w]);
        t += (v.x + v.y) + (v.z + v.w);
    }
    __syncthreads();
    return t;
}

// Inclusive prefix sum over the workgroup in thread order.
template <int NT>
__device__ __forceinline__ uint32_t wg_scan(uint32_t x, uint32_t* wt) {
    static_assert(NT % 256 == 0, "wave totals are read four at a time");
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) wt[w] = x;
    __syncthreads();
    uint32_t base = 0;
#pragma unroll
    for (int q = 0; q < NT / 64; q += 4) {  // every wave total at once, 16-byte reads
        const uint4 t = *reinterpret_cast<const uint4*>(&wt[q]);
        base += (q + 0 < w ? t.x : 0u) + (q + 1 < w ? t.y : 0u) + (q + 2 < w ? t.z : 0u) + (q + 3 < w ? t.w : 0u);
    }
    __syncthreads();
    return x + base;
}

// Histogram into lh (2048 bins, bin = (x - lo) >> s) of the values x of a[0, n)
// with lo <= x <= hi, read by the T threads numbered sub = 0..T-1; 8 loads in
// flight per thread.
template <int T>
__device__ __forceinline__ void strided_hist(const uint32_t* __restrict__ a, uint32_t n, int sub, uint32_t lo,
                                             uint32_t hi, uint32_t s, uint32_t* lh) {
    const uint32_t w = hi - lo;  // x in [lo, hi] iff x - lo <= w (unsigned)
    uint32_t e = (uint32_t)sub;
    for (; e + 7 * T < n; e += 8 * T) {
        uint32_t x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = a[e + T * u] - lo;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (x[u] <= w) atomicAdd(&lh[x[u] >> s], 1u);
    }
    for (; e < n; e += T) {
        const uint32_t x = a[e] - lo;
        if (x <= w) atomicAdd(&lh[x >> s], 1u);
    }
}

template <int NT>
__device__ __forceinline__ void wg_hist(const uint32_t* __restrict__ a, uint32_t n, uint32_t lo, uint32_t hi,
                                        uint32_t s, uint32_t* lh) {
    strided_hist<NT>(a, n, threadIdx.x, lo, hi, s, lh);
}

// After a histogram of [lo, hi] with shift s: narrow [lo, hi] to the bin that
// holds rank r (1-based among the counted values) and make r relative to it.
// Clears lh when `clear`.  Every thread returns with the same lo, hi, r, and
// the return value is the number of values in the chosen bin.
template <int NT>
__device__ uint32_t wg_narrow(uint32_t* lh, uint32_t* wt, uint32_t* part, uint32_t s, uint32_t& lo, uint32_t& hi,
                              uint32_t& r, bool clear = true) {
    constexpr int PER = kMedBins / NT;
    const int tid = threadIdx.x;
    __syncthreads();
    uint32_t loc[PER], sum = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        loc[q] = lh[tid * PER + q];
        if (clear) lh[tid * PER + q] = 0;
        sum += loc[q];
    }
    const uint32_t incl = wg_scan<NT>(sum, wt), excl = incl - sum;
    if (excl < r && r <= incl) {
        uint32_t c = excl;
        for (int q = 0; q < PER; ++q) {
            if (c < r && r <= c + loc[q]) {
                part[0] = (uint32_t)(tid * PER + q);
                part[1] = r - c;
                part[2] = loc[q];
                break;
            }
            c += loc[q];
        }
    }
    __syncthreads();
    const uint64_t nlo = (uint64_t)lo + ((uint64_t)part[0] << s);
    const uint64_t top = nlo + ((uint64_t)1 << s) - 1;
    hi = (uint32_t)(top < (uint64_t)hi ? top : (uint64_t)hi);
    lo = (uint32_t)nlo;
    r = part[1];
    const uint32_t nbin = part[2];
    __syncthreads();
    return nbin;
}

// Exact rank-r value (1-based) among the values in [lo, hi] of a[0, n).
// Expects lh clear; leaves it clear.
template <int NT>
__device__ uint32_t wg_select_array(const uint32_t* __restrict__ a, uint32_t n, uint32_t lo, uint32_t hi, uint32_t r,
                                    uint32_t* lh, uint32_t* wt, uint32_t* part) {
    while (lo < hi) {
        const uint32_t s = shift_for((uint64_t)hi - lo + 1);
        wg_hist<NT>(a, n, lo, hi, s, lh);
        wg_narrow<NT>(lh, wt, part, s, lo, hi, r);
    }
    return lo;
}

// The sample's order statistics (one workgroup of kSelThreads = 1024, exact selects over
// the 8192 sample values; +inf padding ranks last).  exact = 0: the sample
// median is the result; exact = 1: the bracket of the full select (or the
// result, when the sample holds every pair).
__device__ void sample_select_body(const MedView& v, int exact, float* h_out) {
    constexpr int NT = kSelThreads;
    __shared__ uint32_t xs[kMedSample];
    __shared__ uint32_t lh[kMedBins];
    __shared__ __align__(16) uint32_t wt[NT / 64];
    __shared__ uint32_t part[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    SelState* sel = v.sel;
    const int N = v.N;
    if (N < 2 || v.fixed_h > 0.0f) {
        if (tid == 0) {
            const float h = N < 2 ? 1.0f : v.fixed_h;
            sel->h = h;
            sel->m2 = -1.0f;
            sel->mode = kModeDone;
            if (h_out) *h_out = h;
        }
        return;
    }
    const uint64_t P = pair_count(N);
    const bool all = P <= (uint64_t)kMedSample;
    const uint32_t S = all ? (uint32_t)P : (uint32_t)kMedSample;
    uint32_t rank[3];
    rank[1] = (S + 1) / 2;
    const float half = kBracketSigmas * 0.5f / sqrtf((float)S);  // four sigmas of the sample median's rank
    rank[0] = (uint32_t)fmaxf(1.0f, floorf((float)S * (0.5f - half)));
    rank[2] = (uint32_t)fminf((float)S, ceilf((float)S * (0.5f + half)));
    uint32_t mn = 0xffffffffu, mx = 0u;  // range of the sample's (non-NaN) values
    {  // the sample into LDS, all loads in flight
        const uint32_t* g = reinterpret_cast<const uint32_t*>(v.smp);
        uint32_t x[kMedSample / NT];
#pragma unroll
        for (int u = 0; u < kMedSample / NT; ++u) x[u] = g[tid + NT * u];
#pragma unroll
        for (int u = 0; u < kMedSample / NT; ++u) {
            xs[tid + NT * u] = x[u];
            if ((uint32_t)(tid + NT * u) < S && x[u] <= 0x7f800000u) {
                mn = min(mn, x[u]);
                mx = max(mx, x[u]);
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        mn = min(mn, (uint32_t)__shfl_xor(mn, off));
        mx = max(mx, (uint32_t)__shfl_xor(mx, off));
    }
    if (lane == 0) {
        lh[wave] = mn;
        lh[NT / 64 + wave] = mx;
    }
    __syncthreads();
    for (int w = 0; w < NT / 64; ++w) {
        mn = min(mn, lh[w]);
        mx = max(mx, lh[NT / 64 + w]);
    }
    __syncthreads();
    for (int b = tid; b < kMedBins; b += NT) lh[b] = 0;
    __syncthreads();
    if (mn > mx) mn = mx = 0x7f800000u;  // every sample value is NaN
    uint32_t lo0 = 0u, hi2 = 0u, m = 0u;
    if (!exact || all) {
        m = wg_select_array<NT>(xs, kMedSample, mn, mx, rank[1], lh, wt, part);
    } else {
        // bracket ends: the bins of one histogram of the sample's range that
        // hold ranks r0 and r2 (at least as wide as the sample's exact
        // quantiles, by at most a bin, 1/2048 of the range, on each side)
        uint32_t a0 = mn, z0 = mx, r0 = rank[0];
        uint32_t a2 = a0, z2 = z0, r2 = rank[2];
        const uint32_t s1 = shift_for((uint64_t)z0 - a0 + 1);
        wg_hist<NT>(xs, kMedSample, a0, z0, s1, lh);
        wg_narrow<NT>(lh, wt, part, s1, a0, z0, r0, false);
        wg_narrow<NT>(lh, wt, part, s1, a2, z2, r2, true);
        lo0 = a0;
        hi2 = z2;
    }
    if (exact && !all) {  // the passes add into a clear histogram and fresh segment counters
        for (int b = tid; b < kMedBins; b += NT) v.hist[b] = 0;
        for (int g = tid; g < kCandSegs; g += NT) sel->seg[g] = 0;
    }
    if (tid != 0) return;
    if (!exact || all) {
        set_bandwidth(sel, N, m, h_out);
        return;
    }
    sel->lo = lo0;
    sel->hi = hi2;
    sel->rank = (uint32_t)((P + 1) / 2);
    sel->shift = shift_for((uint64_t)hi2 - lo0 + 1);
    sel->overflow = 0;
    sel->mode = kModePass0;
}

// ---- all-pairs work item (row block rb, column chunk cc) ---------------------------
// Pass 0: counts under / over [lo, hi] into cnt[item], in-bracket values into
// the candidate segments.  Mode all: histogram of [lo, hi] (LDS, flushed with
// one atomic per non-empty bin).
//
// 256 threads: ROWS rows and 256 / ROWS column groups (a 64-row item gives each
// wave a quarter of the columns, so small problems still fill the chip).  A
// thread measures four columns at a time (four independent FMA chains, 16-byte
// LDS broadcasts); each distance is summed over the coordinates in order.
template <int DP, int ROWS>
__device__ void med_item(const MedView& v, const float* __restrict__ theta, int rb, int cc) {
    constexpr int NT = 256;
    constexpr int CG = NT / ROWS;       // column groups
    constexpr int CPG = kMedCols / CG;  // columns per group
    constexpr int LD = DP + 4;          // staged row stride: 16-byte aligned rows
    static_assert(NT % ROWS == 0 && CPG % 4 == 0 && ROWS % 64 == 0, "item shape");
    static_assert(kMedCols * DP % NT == 0, "staging covers the columns exactly");
    __shared__ __align__(16) float tj[kMedCols][LD];
    __shared__ uint32_t lh[kMedBins];
    __shared__ uint32_t red[2][NT / 64];
    __shared__ uint32_t wbuf[NT / 64][kWaveBuf];  // each wave's candidates before a flush
    SelState* sel = v.sel;
    const uint32_t mode = sel->mode;
    if (mode != kModePass0 && mode != kModeAll) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int rloc = tid % ROWS, cg = tid / ROWS;
    const int N = v.N, d = v.d;
    const int row0 = rb * ROWS, col0 = cc * kMedCols;
    const bool pass0 = mode == kModePass0;
    uint32_t* cnt = v.cnt + 2 * ((int64_t)rb * v.cc + cc);
    if (col0 + kMedCols <= row0 + 1) {  // no pair i < j in this item
        if (pass0 && tid == 0) cnt[0] = cnt[1] = 0;
        return;
    }
    const uint32_t lo = sel->lo, hi = sel->hi, s = sel->shift;
    if (!pass0)
        for (int b = tid; b < kMedBins; b += NT) lh[b] = 0;
    {  // stage the columns: consecutive threads read consecutive columns
        constexpr int SPT = kMedCols * DP / NT;
        float x[SPT];
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            const int e = tid + NT * u, c = e % kMedCols, l = e / kMedCols;
            const int j = col0 + c;
            x[u] = (j < N && l < d) ? theta[(int64_t)l * N + j] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            const int e = tid + NT * u;
            tj[e % kMedCols][e / kMedCols] = x[u];
        }
    }
    const int i = row0 + rloc;
    float ti[DP];
#pragma unroll
    for (int l = 0; l < DP; ++l) ti[l] = (i < N && l < d) ? theta[(int64_t)l * N + i] : 0.0f;
    __syncthreads();
    // this wave's candidate segment; its candidates gather in wb and go out
    // in one reservation per flush
    const int wave = tid >> 6;
    const int seg = (int)(((blockIdx.y * gridDim.x + blockIdx.x) * (uint32_t)(NT / 64) + (uint32_t)wave) % kCandSegs);
    const uint32_t seg_cap = v.cap / kCandSegs;
    uint32_t* segbuf = v.cand + (size_t)seg * seg_cap;
    uint32_t* wb = wbuf[wave];
    uint32_t nwb = 0;
    const uint64_t lt = (1ull << lane) - 1ull;
    auto flush = [&]() {
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");  // the wave's LDS writes before its reads
        uint32_t base = 0;
        if (lane == 0) {
            base = atomicAdd(&sel->seg[seg], nwb);
            if ((uint64_t)base + nwb > seg_cap) atomicOr(&sel->overflow, 1u);
        }
        base = __shfl(base, 0);
        for (uint32_t e = (uint32_t)lane; e < nwb; e += 64)
            if (base + e < seg_cap) segbuf[base + e] = wb[e];
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");  // reads before the next writes
        nwb = 0;
    };
    uint32_t nb = 0, na = 0;
    // the wave's columns, from the first one past its first row (j > i)
    const int wrow0 = row0 + (rloc & ~63);
    const int cbeg = cg * CPG, cend = cbeg + CPG;
    const int jskip = wrow0 + 1 - col0 - cbeg;
    const int cstart = cbeg + (jskip > 0 ? (jskip & ~3) : 0);
    for (int c = cstart; c < cend; c += 4) {
        float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int l = 0; l < DP; l += 4) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float4 t = *reinterpret_cast<const float4*>(&tj[c + q][l]);
                float df = ti[l] - t.x;
                acc[q] = fmaf(df, df, acc[q]);
                df = ti[l + 1] - t.y;
                acc[q] = fmaf(df, df, acc[q]);
                df = ti[l + 2] - t.z;
                acc[q] = fmaf(df, df, acc[q]);
                df = ti[l + 3] - t.w;
                acc[q] = fmaf(df, df, acc[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = col0 + c + q;
            const bool valid = i < N && j < N && j > i;
            const uint32_t bits = __float_as_uint(acc[q]);
            const bool below = valid && bits < lo;
            const bool above = valid && bits > hi;
            const bool inr = valid && !below && !above;
            if (!pass0) {
                if (inr) atomicAdd(&lh[(bits - lo) >> s], 1u);
                continue;
            }
            nb += below ? 1u : 0u;
            na += above ? 1u : 0u;
            const uint64_t mi = __ballot(inr);
            if (mi) {
                if (nwb + 64 > kWaveBuf) flush();
                if (inr) wb[nwb + (uint32_t)__popcll(mi & lt)] = bits;
                nwb += (uint32_t)__popcll(mi);
            }
        }
    }
    if (!pass0) {
        __syncthreads();
        for (int b = tid; b < kMedBins; b += NT)
            if (lh[b]) atomicAdd(&v.hist[b], lh[b]);
        return;
    }
    if (nwb) flush();
    for (int off = 32; off > 0; off >>= 1) {  // counts of the workgroup
        nb += __shfl_xor(nb, off);
        na += __shfl_xor(na, off);
    }
    if (lane == 0) {
        red[0][tid >> 6] = nb;
        red[1][tid >> 6] = na;
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t b = 0, a = 0;
        for (int w = 0; w < NT / 64; ++w) {
            b += red[0][w];
            a += red[1][w];
        }
        cnt[0] = b;
        cnt[1] = a;
    }
}

// The same item with the distances in Gram form on the FP32 matrix cores:
// D_ij = max(|x_i|^2 + |x_j|^2 - 2 x_i . x_j, 0) over the centred rows the
// FP32 contraction uses (built before the median).  Each wave takes 64 rows
// as four 16-row tiles; with 256-row items it takes every column of the item,
// with 64-row items a 16-column quarter.  Per 16 columns and row tile, KS
// MFMAs (16x16x4) give S[i][j] with lane l holding rows 4 (l / 16) + t of
// column l % 16.  KS = 0 is the split form (d <= 31): the rows as three
// BF16 parts and x_i . x_j as the six part products of order >= 2^-16 on the
// BF16 matrix cores (16x16x32, the same output layout), FP32-accurate as the
// FP32 direction's split form (its rows' slot 31, which holds -|x|^2 / 2's
// parts for the contraction, is zeroed in the row operand).  Every pass computes a pair's distance with
// the same instructions, so the counts stay exact.
// The split form's part products (row part, column part), smallest first.
__device__ constexpr int kGramPairs3[6][2] = {{1, 1}, {2, 0}, {0, 2}, {1, 0}, {0, 1}, {0, 0}};

template <int KS, int ROWS>
__device__ void med_item_gram(const MedView& v, int rb, int cc) {
    // an item spans kGramGroup column chunks: its counts go to the first
    // chunk's slot and zeros to the others
    const int cc1 = min(cc + kGramGroup, v.cc);
    constexpr int NT = 256;
    static_assert(ROWS == 64 || ROWS == 256, "item shape");
    // pass 0 stages candidates per wave, the histogram passes count into lh:
    // one LDS region serves both
    constexpr uint32_t kBuf = 2048;  // flushed when a step (at most 16 x 64 values) might not fit
    // a wave's staging is kBuf words and 64 more, one per lane, that take the
    // stores of the values outside the bracket (the unconditional store)
    constexpr uint32_t kWave = kBuf + 64;
    static_assert(kMedBins <= (NT / 64) * kWave, "histogram inside the staging region");
    __shared__ uint32_t lds_region[(NT / 64) * kWave];
    uint32_t* const lh = lds_region;
    __shared__ uint32_t red[2][NT / 64];
    SelState* sel = v.sel;
    const uint32_t mode = sel->mode;
    if (mode != kModePass0 && mode != kModeAll) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int col = lane & 15, kq = lane >> 4;
    const int N = v.N;
    const int row0 = rb * ROWS, col0 = cc * kMedCols;
    const bool pass0 = mode == kModePass0;
    uint32_t* cnt = v.cnt + 2 * ((int64_t)rb * v.cc + cc);
    if (pass0)
        for (int e = 2 + tid; e < 2 * (cc1 - cc); e += NT) cnt[e] = 0;
    if (cc1 * kMedCols <= row0 + 1) {  // no pair i < j in this item
        if (pass0 && tid == 0) cnt[0] = cnt[1] = 0;
        return;
    }
    const uint32_t lo = sel->lo, hi = sel->hi, s = sel->shift;
    if (!pass0)
        for (int b = tid; b < kMedBins; b += NT) lh[b] = 0;
    __syncthreads();
    const int wrow = ROWS == 256 ? row0 + 64 * wave : row0;
    // 256-row items: every 16-column step for each wave; 64-row items: the
    // waves take the steps in turn
    const int cbeg = ROWS == 256 ? 0 : 16 * wave, cend = (cc1 - cc) * kMedCols, cstep = ROWS == 256 ? 16 : 64;
    constexpr bool SPLIT = KS == 0;
    constexpr int KA = SPLIT ? 1 : KS;   // FP32 operand steps
    constexpr int NP = SPLIT ? 3 : 1;    // split-form parts
    float xa[4][KA];
    bf16x8v xa3[NP][4];
    f4v ni[4];  // |x_i|^2 for i = wrow + 16 r + 4 kq + t
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if constexpr (SPLIT) {
            const __bf16* p = v.xs3 + (int64_t)(wrow + 16 * r + col) * 96 + 8 * kq;
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                xa3[q][r] = *reinterpret_cast<const bf16x8v*>(p + 32 * q);
                if (kq == 3) xa3[q][r][7] = (__bf16)0.0f;  // slot 31 holds e_i's part for the contraction
            }
        } else {
            const float* p = v.xr + (int64_t)(wrow + 16 * r + col) * (4 * KS) + kq * KS;
#pragma unroll
            for (int k = 0; k < KS; ++k) xa[r][k] = p[k];
        }
        ni[r] = *reinterpret_cast<const f4v*>(v.nrm + wrow + 16 * r + 4 * kq);
    }
    // one candidate segment per workgroup (hashed: in a work list only every
    // kGramGroup-th entry runs, and a plain modulus would leave segments unused)
    const int seg = (int)(mix32(blockIdx.y * gridDim.x + blockIdx.x) % kCandSegs);
    const uint32_t seg_cap = v.cap / kCandSegs;
    uint32_t* segbuf = v.cand + (size_t)seg * seg_cap;
    uint32_t* wb = lds_region + wave * kWave;
    uint32_t nwb = 0;
    auto flush = [&]() __attribute__((always_inline)) {
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");  // the wave's LDS writes before its reads
        uint32_t base = 0;
        if (lane == 0) {
            base = atomicAdd(&sel->seg[seg], nwb);
            if ((uint64_t)base + nwb > seg_cap) atomicOr(&sel->overflow, 1u);
        }
        base = __shfl(base, 0);
        for (uint32_t e = (uint32_t)lane; e < nwb; e += 64)
            if (base + e < seg_cap) segbuf[base + e] = wb[e];
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");  // reads before the next writes
        nwb = 0;
    };
    // wave-uniform counts of the wave's valid pairs, of those below lo and of
    // those inside [lo, hi] (a pair is inside iff bits - lo <= hi - lo,
    // unsigned); the pairs above hi are the rest
    uint32_t nvalid = 0, nb = 0, nin = 0;
    uint32_t nbl = 0;  // this lane's pairs below lo on the steps without checks (added to nb at the end)
    const uint32_t wlo = hi - lo;
    // the first step with a pair j > i for some row of the wave; the next
    // step's operands load while this one computes
    int c0 = cbeg;
    while (c0 < cend && col0 + c0 + 15 <= wrow) c0 += cstep;
    float xb[KA], xn[KA];
    bf16x8v xb3[NP], xn3[NP];
    float nj = 0.0f, nn = 0.0f;
    auto load = [&](int c, float (&x)[KA], bf16x8v (&x3)[NP], float& n) __attribute__((always_inline)) {
        if constexpr (SPLIT) {
            const __bf16* p = v.xs3 + (int64_t)(col0 + c + col) * 96 + 8 * kq;
#pragma unroll
            for (int q = 0; q < NP; ++q) x3[q] = *reinterpret_cast<const bf16x8v*>(p + 32 * q);
        } else {
            const float* p = v.xr + (int64_t)(col0 + c + col) * (4 * KS) + kq * KS;
#pragma unroll
            for (int k = 0; k < KS; ++k) x[k] = p[k];
        }
        n = v.nrm[col0 + c + col];
    };
    // one distance of the step: counted, and appended (pass 0) or
    // histogrammed when inside the bracket; ALL: every pair of the step is
    // valid (no row or column checks)
    auto classify = [&](auto all_tag, auto p0_tag, uint32_t x, bool valid) __attribute__((always_inline)) {
        constexpr bool ALL = decltype(all_tag)::value, P0 = decltype(p0_tag)::value;
        if constexpr (ALL && P0) {
            // the common step, without branches: the lane counts its pairs
            // below lo, and every lane stores, an in-bracket value at its
            // compacted place, any other value at the lane's own spare word
            nbl += x < lo ? 1u : 0u;
            const bool inb = x - lo <= wlo;
            const uint64_t mb = __ballot(inb);
            const uint32_t nm = (uint32_t)__popcll(mb);
            const uint32_t pos =
                nwb + __builtin_amdgcn_mbcnt_hi((uint32_t)(mb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mb, 0u));
            wb[inb ? pos : kBuf + (uint32_t)lane] = x;
            nin += nm;
            nwb = __builtin_amdgcn_readfirstlane(nwb + nm);
            return;
        }
        const bool in = (ALL || valid) && x - lo <= wlo;
        if (P0) {
            nb += (uint32_t)__popcll(__ballot((ALL || valid) && x < lo));
            if (!ALL) nvalid += (uint32_t)__popcll(__ballot(valid));
        }
        const uint64_t m = __ballot(in);
        if (m) {
            if (P0) {
                const uint32_t nm = (uint32_t)__popcll(m);
                nin += nm;
                const uint32_t pos =
                    nwb + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                if (in) wb[pos] = x;
                nwb = __builtin_amdgcn_readfirstlane(nwb + nm);  // uniform: keep it scalar
            } else if (in) {
                atomicAdd(&lh[(x - lo) >> s], 1u);
            }
        }
    };
    auto sweep = [&](auto p0_tag) __attribute__((always_inline)) {
        constexpr bool P0 = decltype(p0_tag)::value;
        if (c0 < cend) load(c0, xb, xb3, nj);
        for (int c = c0; c < cend; c += cstep) {
            if (c + cstep < cend) load(c + cstep, xn, xn3, nn);
            const int jb = col0 + c, j = jb + col;
            // a step appends at most 16 x 64 values
            if (P0 && nwb + 1024 > kBuf) flush();
            uint32_t bv[16];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                f4v S = f4v{0.f, 0.f, 0.f, 0.f};
                if constexpr (SPLIT) {
#pragma unroll
                    for (int e = 0; e < 6; ++e)
                        S = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa3[kGramPairs3[e][0]][r], xb3[kGramPairs3[e][1]],
                                                                    S, 0, 0, 0);
                } else {
#pragma unroll
                    for (int k = 0; k < KS; ++k) S = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[r][k], xb[k], S, 0, 0, 0);
                }
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    bv[4 * r + t] = __float_as_uint(fmaxf(fmaf(-2.0f, S[t], ni[r][t] + nj), 0.0f));
            }
            if constexpr (SPLIT) {
#pragma unroll
                for (int q = 0; q < NP; ++q) xb3[q] = xn3[q];
            } else {
#pragma unroll
                for (int k = 0; k < KS; ++k) xb[k] = xn[k];
            }
            nj = nn;
            if (jb > wrow + 63 && jb + 16 <= N) {  // wave-uniform
#pragma unroll
                for (int e = 0; e < 16; ++e) classify(std::true_type{}, p0_tag, bv[e], true);
                nvalid += 1024;
            } else {
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int i = wrow + 16 * (e >> 2) + 4 * kq + (e & 3);
                    classify(std::false_type{}, p0_tag, bv[e], i < N && j < N && j > i);
                }
            }
        }
    };
    if (pass0) {
        sweep(std::true_type{});
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) nbl += __shfl_xor(nbl, o);
        nb += __builtin_amdgcn_readfirstlane(nbl);
    } else {
        sweep(std::false_type{});
    }
    if (!pass0) {
        __syncthreads();
        for (int b = tid; b < kMedBins; b += NT)
            if (lh[b]) atomicAdd(&v.hist[b], lh[b]);
        return;
    }
    // the workgroup's remaining candidates go out under one reservation (the
    // segment counters are shared by every workgroup: one atomic each)
    __shared__ uint32_t wn[NT / 64 + 1];
    if (lane == 0) wn[wave] = nwb;
    __syncthreads();
    if (tid == 0) {
        const uint32_t tot = wn[0] + wn[1] + wn[2] + wn[3];
        uint32_t base = 0;
        if (tot) {
            base = atomicAdd(&sel->seg[seg], tot);
            if ((uint64_t)base + tot > seg_cap) atomicOr(&sel->overflow, 1u);
        }
        wn[NT / 64] = base;
    }
    __syncthreads();
    {
        uint32_t off = wn[NT / 64];
        for (int w = 0; w < wave; ++w) off += wn[w];
        for (uint32_t e = (uint32_t)lane; e < nwb; e += 64)
            if (off + e < seg_cap) segbuf[off + e] = wb[e];
    }
    if (lane == 0) {  // counts of the workgroup
        red[0][wave] = nb;
        red[1][wave] = nvalid - nb - nin;
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t b = 0, a = 0;
        for (int w = 0; w < NT / 64; ++w) {
            b += red[0][w];
            a += red[1][w];
        }
        cnt[0] = b;
        cnt[1] = a;
    }
}

// Candidate pass: histogram of the candidates in [lo, hi] (sentinels and
// values outside are skipped); segment g, part `part` of kCandParts.
__device__ void med_cand_body(const MedView& v, int g, int part) {
    __shared__ uint32_t lh[kMedBins];
    const SelState* sel = v.sel;
    if (sel->mode != kModeCand) return;
    const uint32_t lo = sel->lo, hi = sel->hi, s = sel->shift;
    const uint32_t seg_cap = v.cap / kCandSegs;
    const uint32_t n = sel->seg[g] < seg_cap ? sel->seg[g] : seg_cap;
    const uint32_t* segbuf = v.cand + (size_t)g * seg_cap;
    for (int b = threadIdx.x; b < kMedBins; b += 256) lh[b] = 0;
    __syncthreads();
    const uint32_t per = (n + kCandParts - 1) / kCandParts;  // this part's slice of the segment
    const uint32_t b0 = (uint32_t)part * per;
    if (b0 < n) wg_hist<256>(segbuf + b0, (b0 + per < n ? per : n - b0), lo, hi, s, lh);
    __syncthreads();
    for (int b = threadIdx.x; b < kMedBins; b += 256)
        if (lh[b]) atomicAdd(&v.hist[b], lh[b]);
}

// Select step (one workgroup of 256).  After pass 0: is rank k under, in or
// over the bracket?  After a histogram pass: the bin holding the rank.  The
// histogram is cleared for the next pass; h is set once the interval is one
// value.
__device__ void med_select_body(const MedView& v, float* h_out) {
    constexpr int PER = kMedBins / 256;
    __shared__ uint32_t psum[256];
    __shared__ uint32_t tot[2];
    const int tid = threadIdx.x;
    SelState* sel = v.sel;
    const uint32_t mode = sel->mode;
    if (mode == kModeDone) return;
    const uint32_t lo = sel->lo, hi = sel->hi, s = sel->shift;
    const uint32_t r = sel->rank;
    if (mode == kModePass0) {
        // sum the items' counts in a fixed order, sixteen 8-byte loads in
        // flight per thread (this step waits on memory, often beside a
        // bandwidth-bound rollout)
        const int items = v.rb * v.cc;
        const uint2* cnt2 = reinterpret_cast<const uint2*>(v.cnt);
        uint32_t cb = 0, ca = 0;
        for (int e = tid; e < items; e += 256 * 16) {
            uint2 q[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) q[u] = cnt2[min(e + 256 * u, items - 1)];
#pragma unroll
            for (int u = 0; u < 16; ++u)
                if (e + 256 * u < items) {
                    cb += q[u].x;
                    ca += q[u].y;
                }
        }
        for (int k = 0; k < 2; ++k) {
            psum[tid] = k == 0 ? cb : ca;
            __syncthreads();
            for (int w = 128; w > 0; w >>= 1) {
                if (tid < w) psum[tid] += psum[tid + w];
                __syncthreads();
            }
            if (tid == 0) tot[k] = psum[0];
            __syncthreads();
        }
        if (tid == 0) {
            const uint32_t below = tot[0], above = tot[1];
            const uint32_t inside = (uint32_t)(pair_count(v.N) - below - above);
            if (r <= below) {  // under the bracket: every pair again over [0, lo - 1]
                sel->hi = lo - 1;
                sel->lo = 0;
                sel->shift = shift_for((uint64_t)lo);
                sel->mode = kModeAll;
            } else if (r > below + inside) {  // over it: over [hi + 1, 0xffffffff]
                sel->rank = r - below - inside;
                sel->lo = hi + 1;
                sel->hi = 0xffffffffu;
                sel->shift = shift_for((uint64_t)0xffffffffu - hi);
                sel->mode = kModeAll;
            } else {
                sel->rank = r - below;
                sel->mode = sel->overflow ? kModeAll : kModeCand;
            }
        }
        return;
    }
    uint32_t loc[PER];
    uint32_t sum = 0;
    for (int q = 0; q < PER; ++q) {
        loc[q] = v.hist[tid * PER + q];
        v.hist[tid * PER + q] = 0;
        sum += loc[q];
    }
    psum[tid] = sum;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {  // inclusive scan
        const uint32_t x = tid >= off ? psum[tid - off] : 0;
        __syncthreads();
        psum[tid] += x;
        __syncthreads();
    }
    const uint32_t incl = psum[tid], excl = incl - sum;
    if (excl < r && r <= incl) {
        uint32_t c = excl;
        for (int q = 0; q < PER; ++q) {
            if (c < r && r <= c + loc[q]) {
                const uint64_t nlo = (uint64_t)lo + ((uint64_t)(tid * PER + q) << s);
                const uint64_t top = nlo + ((uint64_t)1 << s) - 1;
                const uint64_t nhi = top < (uint64_t)hi ? top : (uint64_t)hi;
                sel->rank = r - c;
                sel->lo = (uint32_t)nlo;
                sel->hi = (uint32_t)nhi;
                if (nlo == nhi) set_bandwidth(sel, v.N, (uint32_t)nlo, h_out);
                else sel->shift = shift_for(nhi - nlo + 1);
                break;
            }
            c += loc[q];
        }
    }
}


// Small problems (P <= kFinishPairs): everything after pass 0 in one
// workgroup of kFinishThreads.  The counts decide where rank k lies.  Inside
// the bracket (and without overflow) the candidates are read into registers
// once and histogram passes over them narrow the interval (two, for the usual
// bracket width).  Else (rare) histogram passes run over every pair,
// recomputed here.
constexpr uint64_t kFinishPairs = 1ull << 20;

// Problems above kFinishPairs pairs take the Gram-form distances in their
// all-pairs passes (when the caller provides the operands); smaller ones keep
// direct differences, in the single-problem and the batched paths alike, so
// both reach the same bandwidth bit for bit.
__host__ __device__ __forceinline__ bool med_gram(int N) { return pair_count(N) > kFinishPairs; }
constexpr int kFinishThreads = 1024;
constexpr int kFinishRegs = 40;         // candidate slots per thread held in registers
constexpr int kSegThreads = kFinishThreads / kCandSegs;
static_assert(kFinishThreads % kCandSegs == 0, "whole thread groups per candidate segment");

__device__ void med_finish_body(const MedView& v, const float* __restrict__ theta, float* h_out) {
    constexpr int NT = kFinishThreads;
    __shared__ uint32_t lh[kMedBins];
    __shared__ __align__(16) uint32_t wt[NT / 64];
    __shared__ uint32_t part[4];
    const int tid = threadIdx.x;
    SelState* sel = v.sel;
    if (sel->mode != kModePass0) return;
    const int N = v.N, d = v.d;
    uint32_t lo = sel->lo, hi = sel->hi;
    uint32_t r = sel->rank;
    uint32_t b = 0, a = 0;
    for (int e = tid; e < v.rb * v.cc; e += NT) {
        b += v.cnt[2 * e];
        a += v.cnt[2 * e + 1];
    }
    const uint32_t below = wg_sum<NT>(b, wt), above = wg_sum<NT>(a, wt);
    const uint32_t inside = (uint32_t)(pair_count(N) - below - above);
    for (int q = tid; q < kMedBins; q += NT) lh[q] = 0;
    __syncthreads();
    if (r > below && r <= below + inside && !sel->overflow) {
        // select among the candidates in [lo, hi] (sentinels lie above hi)
        r -= below;
        const uint32_t seg_cap = v.cap / kCandSegs;
        const int g = tid / kSegThreads, sub = tid % kSegThreads;
        const uint32_t n = sel->seg[g] < seg_cap ? sel->seg[g] : seg_cap;
        const uint32_t* sb = v.cand + (size_t)g * seg_cap;
        // the first kFinishRegs * kSegThreads slots of each segment stay in
        // registers (one load round trip); longer segments stream the rest
        constexpr uint32_t nreg = kFinishRegs * kSegThreads;
        // slots past n lie inside the segment (at least kCandSegMin slots) and
        // read as sentinels
        static_assert(kFinishRegs * kSegThreads <= (int)kCandSegMin, "register slots inside every segment");
        uint32_t xr[kFinishRegs];
#pragma unroll
        for (int u = 0; u < kFinishRegs; ++u) xr[u] = sb[sub + kSegThreads * u];
#pragma unroll
        for (int u = 0; u < kFinishRegs; ++u)
            if ((uint32_t)(sub + kSegThreads * u) >= n) xr[u] = kSentinel;
        auto hist_pass = [&](uint32_t s) {
            const uint32_t w = hi - lo;
#pragma unroll
            for (int u = 0; u < kFinishRegs; ++u) {
                const uint32_t dx = xr[u] - lo;  // in [lo, hi] iff dx <= hi - lo (unsigned)
                if (dx <= w) atomicAdd(&lh[dx >> s], 1u);
            }
            if (n > nreg) strided_hist<kSegThreads>(sb + nreg, n - nreg, sub, lo, hi, s, lh);
        };
        while (lo < hi) {  // each pass narrows the width 2048-fold: two passes, usually
            const uint32_t s = shift_for((uint64_t)hi - lo + 1);
            hist_pass(s);
            wg_narrow<NT>(lh, wt, part, s, lo, hi, r);
        }
        if (tid == 0) set_bandwidth(sel, N, lo, h_out);
        return;
    }
    if (r <= below) {
        hi = lo - 1;
        lo = 0;
    } else if (r > below + inside) {
        r -= below + inside;
        lo = hi + 1;
        hi = 0xffffffffu;
    } else {
        r -= below;  // inside, but the candidates overflowed
    }
    while (lo < hi) {  // histogram passes over every pair (rare)
        const uint32_t s = shift_for((uint64_t)hi - lo + 1);
        for (int i = tid; i < N; i += NT)
            for (int j = i + 1; j < N; ++j) {
                float acc = 0.0f;
                for (int l = 0; l < d; ++l) {
                    const float df = theta[(int64_t)l * N + i] - theta[(int64_t)l * N + j];
                    acc = fmaf(df, df, acc);
                }
                const uint32_t x = __float_as_uint(acc);
                if (x >= lo && x <= hi) atomicAdd(&lh[(x - lo) >> s], 1u);
            }
        wg_narrow<NT>(lh, wt, part, s, lo, hi, r);
    }
    if (tid == 0) set_bandwidth(sel, N, lo, h_out);
}

// ---- single-problem kernels -----------------------------------------------------
struct OneMed {
    int N, d;
    float fixed_h;
    SvgdLayout L;
    char* ws;
};

// four lanes per sample slot
__global__ __launch_bounds__(256) void k_med_dist(OneMed a, const float* theta) {
    if (a.N < 2 || a.fixed_h > 0.0f) return;
    const int t = blockIdx.x * 64 + (threadIdx.x >> 2), q = threadIdx.x & 3;
    const float v = sample_dist4(a.N, a.d, t, q, theta);
    if (q == 0) med_view(a.N, a.d, a.fixed_h, a.L, a.ws).smp[t] = v;
}

__global__ __launch_bounds__(kSelThreads) void k_sample_select(OneMed a, int exact, float* h_out) {
    sample_select_body(med_view(a.N, a.d, a.fixed_h, a.L, a.ws), exact, h_out);
}

template <int DP, int ROWS>
__global__ __launch_bounds__(256) void k_med_items(OneMed a, const float* theta) {
    med_item<DP, ROWS>(med_view(a.N, a.d, a.fixed_h, a.L, a.ws), theta, blockIdx.y, blockIdx.x);
}

template <int KS, int ROWS>
__global__ __launch_bounds__(256) void k_med_items_gram(OneMed a) {
    med_item_gram<KS, ROWS>(med_view(a.N, a.d, a.fixed_h, a.L, a.ws), blockIdx.y, blockIdx.x * kGramGroup);
}

__global__ __launch_bounds__(256) void k_med_cand(OneMed a) {
    med_cand_body(med_view(a.N, a.d, a.fixed_h, a.L, a.ws), blockIdx.x / kCandParts, blockIdx.x % kCandParts);
}

__global__ __launch_bounds__(256) void k_med_select(OneMed a, float* h_out) {
    med_select_body(med_view(a.N, a.d, a.fixed_h, a.L, a.ws), h_out);
}

__global__ __launch_bounds__(kFinishThreads) void k_med_finish(OneMed a, const float* theta, float* h_out) {
    med_finish_body(med_view(a.N, a.d, a.fixed_h, a.L, a.ws), theta, h_out);
}

// ---- batched kernels ---------------------------------------------------------------
__device__ __forceinline__ MedView med_of(const ProblemDesc& D, char* ws) {
    return med_view(D.N, D.d, D.fixed_h, D.sv, ws + D.svgd_off);
}

// grid (kMedSample / 64, problems): four lanes per sample slot
__global__ __launch_bounds__(256) void k_med_dist_batched(const ProblemDesc* __restrict__ descs, const float* theta,
                                                          char* ws) {
    const ProblemDesc& D = descs[blockIdx.y];
    if (D.N < 2 || D.fixed_h > 0.0f) return;
    const int t = blockIdx.x * 64 + (threadIdx.x >> 2), q = threadIdx.x & 3;
    const float v = sample_dist4(D.N, D.d, t, q, theta + D.theta_off);
    if (q == 0) med_of(D, ws).smp[t] = v;
}

__global__ __launch_bounds__(kSelThreads) void k_sample_select_batched(const ProblemDesc* __restrict__ descs, char* ws,
                                                                int exact) {
    sample_select_body(med_of(descs[blockIdx.x], ws), exact, nullptr);
}

// The BF16 form's bandwidth stage in two launches.  First: blocks below
// nd = (kMedSample / 64) x problems gather the sample distances (four lanes a
// slot), the rest take one entry (problem, coordinate) of the centre list
// each.  Second: one workgroup per problem selects the sample median (the
// scaled rows, which need it, are packed with V).  A non-null step counter is
// advanced once by the first launch (a solve's iteration counter, read by
// the update at the iteration's end).
__global__ __launch_bounds__(256) void k_bw16_gather_batched(const ProblemDesc* __restrict__ descs,
                                                             const int4* __restrict__ ctr_work, int nd,
                                                             const float* theta, char* ws, int* step) {
    constexpr int per = kMedSample / 64;
    if (step && blockIdx.x == 0 && threadIdx.x == 0) *step += 1;
    if ((int)blockIdx.x < nd) {
        const ProblemDesc& D = descs[blockIdx.x / per];
        if (D.N < 2 || D.fixed_h > 0.0f) return;
        const int t = (blockIdx.x % per) * 64 + (threadIdx.x >> 2), q = threadIdx.x & 3;
        const float v = sample_dist4(D.N, D.d, t, q, theta + D.theta_off);
        if (q == 0) med_of(D, ws).smp[t] = v;
        return;
    }
    const int4 e = ctr_work[blockIdx.x - nd];
    const ProblemDesc& D = descs[e.x];
    particle_mean_body<kCentreThreads>(D.N, e.y, theta + D.theta_off,
                                       reinterpret_cast<float*>(ws + D.svgd_off + D.sv.ctr_off));
}

// entry = (problem, row block, column chunk, -) of this item shape's work list
template <int DP, int ROWS>
__global__ __launch_bounds__(256) void k_med_items_batched(const ProblemDesc* __restrict__ descs,
                                                            const int4* __restrict__ work, const float* theta,
                                                            char* ws) {
    const int4 w = work[blockIdx.x];
    const ProblemDesc& D = descs[w.x];
    med_item<DP, ROWS>(med_of(D, ws), theta + D.theta_off, w.y, w.z);
}

template <int KS, int ROWS>
__global__ __launch_bounds__(256) void k_med_items_gram_batched(const ProblemDesc* __restrict__ descs,
                                                                 const int4* __restrict__ work, char* ws) {
    const int4 w = work[blockIdx.x];
    const ProblemDesc& D = descs[w.x];
    // the entry that starts a group of kGramGroup column chunks runs them all
    if (w.z % kGramGroup != 0) return;
    med_item_gram<KS, ROWS>(med_of(D, ws), w.y, w.z);
}

// entry = (problem, segment, part, -)
__global__ __launch_bounds__(256) void k_med_cand_batched(const ProblemDesc* __restrict__ descs,
                                                          const int4* __restrict__ work, char* ws) {
    const int4 w = work[blockIdx.x];
    med_cand_body(med_of(descs[w.x], ws), w.y, w.z);
}

__global__ __launch_bounds__(256) void k_med_select_batched(const ProblemDesc* __restrict__ descs, char* ws) {
    med_select_body(med_of(descs[blockIdx.x], ws), nullptr);
}

// entry = (problem, -, -, -) of a problem of 2^20 pairs at most: the select
// ends in one workgroup after pass 0, as in the single-problem path
__global__ __launch_bounds__(kFinishThreads) void k_med_finish_batched(const ProblemDesc* __restrict__ descs,
                                                                       const int4* __restrict__ work,
                                                                       const float* theta, char* ws) {
    const ProblemDesc& D = descs[work[blockIdx.x].x];
    med_finish_body(med_of(D, ws), theta + D.theta_off, nullptr);
}

template <int ROWS>
void launch_items_rows(const OneMed& a, const float* theta, hipStream_t st) {
    const dim3 grid(a.L.med_cc, a.L.med_rb);
    const int dp = med_dp(a.d);
    if (dp == 16) hipLaunchKernelGGL((k_med_items<16, ROWS>), grid, dim3(256), 0, st, a, theta);
    else if (dp == 32) hipLaunchKernelGGL((k_med_items<32, ROWS>), grid, dim3(256), 0, st, a, theta);
    else hipLaunchKernelGGL((k_med_items<64, ROWS>), grid, dim3(256), 0, st, a, theta);
}

void launch_items(const OneMed& a, const float* theta, hipStream_t st) {
    if (a.L.med_rows == 64) launch_items_rows<64>(a, theta, st);
    else launch_items_rows<256>(a, theta, st);
}

template <int KS>
void launch_items_gram_ks(const OneMed& a, hipStream_t st) {
    const dim3 grid((a.L.med_cc + kGramGroup - 1) / kGramGroup, a.L.med_rb);
    if (a.L.med_rows == 64) hipLaunchKernelGGL((k_med_items_gram<KS, 64>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_med_items_gram<KS, 256>), grid, dim3(256), 0, st, a);
}

void launch_items_gram(const OneMed& a, hipStream_t st) {
    if (a.L.split3) {
        launch_items_gram_ks<0>(a, st);
        return;
    }
    switch (a.L.ks32) {
        case 2: launch_items_gram_ks<2>(a, st); break;
        case 4: launch_items_gram_ks<4>(a, st); break;
        case 6: launch_items_gram_ks<6>(a, st); break;
        case 8: launch_items_gram_ks<8>(a, st); break;
        case 10: launch_items_gram_ks<10>(a, st); break;
        case 12: launch_items_gram_ks<12>(a, st); break;
        case 14: launch_items_gram_ks<14>(a, st); break;
        default: launch_items_gram_ks<16>(a, st); break;
    }
}

// each item shape's work list, in its own launch
template <int DP, int ROWS>
void launch_direct_list(const BatchPlan& P, const ProblemDesc* descs, const float* theta, char* ws, hipStream_t st) {
    const int c = med_class(DP, ROWS);
    if (P.dist_n[c])
        hipLaunchKernelGGL((k_med_items_batched<DP, ROWS>), dim3(P.dist_n[c]), dim3(256), 0, st, descs,
                           P.dist_work + P.dist_start[c], theta, ws);
}

template <int KS>
void launch_gram_lists(const BatchPlan& P, const ProblemDesc* descs, char* ws, hipStream_t st) {
    const int c64 = med_gram_list(KS, 64), c256 = med_gram_list(KS, 256);
    if (P.dist_n[c64])
        hipLaunchKernelGGL((k_med_items_gram_batched<KS, 64>), dim3(P.dist_n[c64]), dim3(256), 0, st, descs,
                           P.dist_work + P.dist_start[c64], ws);
    if (P.dist_n[c256])
        hipLaunchKernelGGL((k_med_items_gram_batched<KS, 256>), dim3(P.dist_n[c256]), dim3(256), 0, st, descs,
                           P.dist_work + P.dist_start[c256], ws);
}

void launch_items_batched(const BatchPlan& P, const ProblemDesc* descs, const float* theta, char* ws,
                          hipStream_t st) {
    if (!P.n_dist) return;
    launch_direct_list<16, 64>(P, descs, theta, ws, st);
    launch_direct_list<32, 64>(P, descs, theta, ws, st);
    launch_direct_list<64, 64>(P, descs, theta, ws, st);
    launch_direct_list<16, 256>(P, descs, theta, ws, st);
    launch_direct_list<32, 256>(P, descs, theta, ws, st);
    launch_direct_list<64, 256>(P, descs, theta, ws, st);
    launch_gram_lists<0>(P, descs, ws, st);
    launch_gram_lists<2>(P, descs, ws, st);
    launch_gram_lists<4>(P, descs, ws, st);
    launch_gram_lists<6>(P, descs, ws, st);
    launch_gram_lists<8>(P, descs, ws, st);
    launch_gram_lists<10>(P, descs, ws, st);
    launch_gram_lists<12>(P, descs, ws, st);
    launch_gram_lists<14>(P, descs, ws, st);
    launch_gram_lists<16>(P, descs, ws, st);
}

}  // namespace

hipError_t launch_median(int N, int d, const float* theta, float bandwidth, int exact, void* ws, const SvgdLayout& L,
                         float* h_out, hipStream_t st, int gram) {
    OneMed a{N, d, bandwidth > 0.0f ? bandwidth : 0.0f, L, static_cast<char*>(ws)};
    // the sample distances only when a median is wanted: with a given
    // bandwidth (or one particle) the select just records h
    if (N >= 2 && !(bandwidth > 0.0f))
        hipLaunchKernelGGL(k_med_dist, dim3(kMedSample / 64), dim3(256), 0, st, a, theta);
    hipLaunchKernelGGL(k_sample_select, dim3(1), dim3(kSelThreads), 0, st, a, exact, h_out);
    if (exact && N >= 2 && !(bandwidth > 0.0f) && pair_count(N) > (uint64_t)kMedSample) {
        // pass 0; small problems keep direct differences, whose every-pair
        // fallback lives in the finishing workgroup
        const bool small = !med_gram(N);
        if (gram && !small) launch_items_gram(a, st);
        else launch_items(a, theta, st);
        if (small) {  // one workgroup finishes
            hipLaunchKernelGGL(k_med_finish, dim3(1), dim3(kFinishThreads), 0, st, a, theta, h_out);
            return hipGetLastError();
        }
        hipLaunchKernelGGL(k_med_select, dim3(1), dim3(256), 0, st, a, h_out);
        for (int pass = 0; pass < 3; ++pass) {
            hipLaunchKernelGGL(k_med_cand, dim3(kCandSegs * kCandParts), dim3(256), 0, st, a);
            if (gram) launch_items_gram(a, st);
            else launch_items(a, theta, st);
            hipLaunchKernelGGL(k_med_select, dim3(1), dim3(256), 0, st, a, h_out);
        }
    }
    return hipGetLastError();
}

hipError_t launch_bandwidth16_batched(const BatchPlan& P, const ProblemDesc* descs, const float* theta, char* ws,
                                      hipStream_t st, int* step) {
    const int np = P.n_problems, nd = (kMedSample / 64) * np;
    hipLaunchKernelGGL(k_bw16_gather_batched, dim3(nd + P.n_ctr), dim3(256), 0, st, descs, P.ctr_work, nd, theta, ws,
                       step);
    hipLaunchKernelGGL(k_sample_select_batched, dim3(np), dim3(kSelThreads), 0, st, descs, ws, 0);
    return hipGetLastError();
}

hipError_t launch_median_batched(const BatchPlan& P, const ProblemDesc* descs, const float* theta, int exact,
                                 char* ws, hipStream_t st) {
    const int np = P.n_problems;
    hipLaunchKernelGGL(k_med_dist_batched, dim3(kMedSample / 64, np), dim3(256), 0, st, descs, theta, ws);
    hipLaunchKernelGGL(k_sample_select_batched, dim3(np), dim3(kSelThreads), 0, st, descs, ws, exact);
    if (exact && P.n_dist) {
        auto items = [&]() { launch_items_batched(P, descs, theta, ws, st); };
        items();
        // problems of 2^20 pairs at most end in one workgroup each; the larger
        // ones take the select and the candidate passes (which skip the
        // problems already done)
        if (P.n_fin)
            hipLaunchKernelGGL(k_med_finish_batched, dim3(P.n_fin), dim3(kFinishThreads), 0, st, descs, P.fin_work,
                               theta, ws);
        if (P.n_cand) {
            hipLaunchKernelGGL(k_med_select_batched, dim3(np), dim3(256), 0, st, descs, ws);
            for (int pass = 0; pass < 3; ++pass) {
                hipLaunchKernelGGL(k_med_cand_batched, dim3(P.n_cand), dim3(256), 0, st, descs, P.cand_work, ws);
                items();
                hipLaunchKernelGGL(k_med_select_batched, dim3(np), dim3(256), 0, st, descs, ws);
            }
        }
    }
    return hipGetLastError();
}

}  // namespace stamp
