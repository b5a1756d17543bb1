// FP32 SVGD direction on the matrix cores (v_mfma_f32_16x16x4f32), the
// contraction of Eq. (1) (Eq. (4) with importance weights):
//
//   x_i = theta_i - mean theta                  (FP32; centring shrinks the Gram cancellation)
//   D_ij = |x_i|^2 + |x_j|^2 - 2 x_i . x_j      (Gram on MFMA, FP32)
//   K_ij = exp(-max(D_ij, 0) / h)
//   V_j = w_j [ g_j - (2/h) x_j | 1 ]           (w_j = 1 without weights)
//   A_i = sum_j K_ij V_j                         (MFMA, FP32)
//   phi_i = ( A_i[0..d) + (2/h) x_i A_i[d] ) / N
//
// which is (1/N) sum_j w_j K_ij [g_j + (2/h)(theta_i - theta_j)] with
// theta_i - theta_j = x_i - x_j.  With c = -log2(e) / h, log2 K_ij =
// -2c (x_i . x_j + e_j) + c |x_i|^2 for e_j = -|x_j|^2 / 2: e_j enters as the
// Gram MFMA's accumulator input, the rest is one fused multiply-add, and the
// exponential's clamp to [0, 1] is the max(D, 0) (one multiply-add and one
// exponential per pair: the VALU work shares the issue port with the MFMAs).
//
// Stages: everything that depends on theta only runs with the median (the
// bandwidth stage, which can overlap the rollout): the particle mean and the
// centred rows in the MFMA operand order with their norms (the median's
// all-pairs passes take their Gram-form distances from these).  The direction
// stage packs V = w [g - (2/h) x | 1 | 0] chunk-tiled from theta, g and the
// weights, so the contraction's loop only loads it; the contraction (64, 128
// or 256 rows per workgroup, 64 per wave as four 16-row tiles, one column
// split) runs per 16 columns the Gram MFMAs of every row tile, turns
// them into K in registers and feeds K as the A operand of the K.V MFMAs: the
// Gram output (lane holds columns j = 4(l/16)+t of row l%16) is an A operand
// whose k index runs over (l/16, t), and V is stored in that order, so each
// lane reads its four V values of an output tile with one 16-byte load.  The
// reduce sums the splits in a fixed order.  Splits depend on N only.
//
// Split form (d <= 31).  The FP32 matrix cores do a sixteenth of the BF16
// ones' work per cycle, so the same contraction runs there with every FP32
// operand v written as three BF16 parts, hi = bf16(v), mid = bf16(v - hi),
// lo = bf16(v - hi - mid) (both differences exact in FP32, and
// hi + mid + lo = v exactly for normal v: 24 significant bits, 8 per part).
// A product a b is then the sum of the six part products whose order is at
// least 2^-16 of it (hh, hm, mh, hl, lh, mm; the three dropped ones are
// below 2^-24, the only error besides the sums), each exact in the FP32
// accumulator: the Gram x_i . x_j takes six BF16 MFMAs over 32 coordinates,
// K V six over 32 particles, where the FP32 form takes eight 4-wide ones and
// eight.  e_j enters through the Gram's spare slot 31 (d <= 31): its three
// parts in the column operand against (1, 0, 0) in the row operand's slot.
// K is the same multiply-add and clamped exponential of the Gram value, so
// the result is the FP32 form's within its own rounding.  Tiling as in the BF16
// direction (phi16.hip): a workgroup of 4 waves owns 64 rows and one column
// split, the waves take its quarters and add their sums through LDS; the
// Gram's output layout is the K.V product's A operand, V is stored in that
// permuted order.  The rows' parts are packed in the bandwidth stage (the
// median's Gram form reads them too), V's after the gradient.  The reduce is
// the FP32 form's.
#include <math.h>

#include <type_traits>

#include "common.h"
#include "internal.h"

namespace stamp {

namespace {

typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f4;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;

struct View32 {  // one problem's FP32 matrix-core workspace
    const float* ctr;
    float* xr;   // [npad][4 ks]: row i, lane group q holds coordinates q ks .. q ks + ks - 1
    float* nrm;  // [npad]: |x_i|^2
    float* vt;   // [npad / 16][ot][16 columns n][16 rows j]: X[j][16 o + n] at 16 n + j of tile (j/16, o)
    float* part; // [splits32][16 ot][npad]
    __bf16* xs3; // split form: [npad][3][32], row i's part p at (3 i + p) 32 (slot 31: -|x_i|^2 / 2's part)
    __bf16* vs3; // split form: part p of V at p npad 16 ot, as [npad / 32][16 ot][32] in MFMA k order
    const SelState* sel;
};

__device__ __forceinline__ View32 view32(const SvgdLayout& L, char* base) {
    View32 v;
    v.ctr = reinterpret_cast<const float*>(base + L.ctr_off);
    v.xr = reinterpret_cast<float*>(base + L.x32_off);
    v.nrm = reinterpret_cast<float*>(base + L.n32_off);
    v.vt = reinterpret_cast<float*>(base + L.v32_off);
    v.part = reinterpret_cast<float*>(base + L.part_off);
    v.xs3 = reinterpret_cast<__bf16*>(base + L.xs3_off);
    v.vs3 = reinterpret_cast<__bf16*>(base + L.vs3_off);
    v.sel = reinterpret_cast<const SelState*>(base + L.sel_off);
    return v;
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef uint32_t u4v __attribute__((ext_vector_type(4)));

// Two values as packed BF16 pairs (element 0 in the low half): one
// conversion, and the pair's values back in FP32 by shift and mask.
__device__ __forceinline__ uint32_t bf16_pair(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f2v{a, b}, bf16x2));
}
__device__ __forceinline__ float pair_lo(uint32_t p) { return __uint_as_float(p << 16); }
__device__ __forceinline__ float pair_hi(uint32_t p) { return __uint_as_float(p & 0xffff0000u); }

// v[u] = hi[u] + mid[u] + lo[u] for eight values (BF16 parts; the two
// differences are exact in FP32)
__device__ __forceinline__ void split3(const float (&v)[8], bf16x8& hi, bf16x8& mid, bf16x8& lo) {
    u4v h, m, l;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        h[q] = bf16_pair(v[2 * q], v[2 * q + 1]);
        const float ra = v[2 * q] - pair_lo(h[q]), rb = v[2 * q + 1] - pair_hi(h[q]);
        m[q] = bf16_pair(ra, rb);
        l[q] = bf16_pair(ra - pair_lo(m[q]), rb - pair_hi(m[q]));
    }
    hi = __builtin_bit_cast(bf16x8, h);
    mid = __builtin_bit_cast(bf16x8, m);
    lo = __builtin_bit_cast(bf16x8, l);
}

// ---- operands: 64 rows per 256 threads, lane group q = threadIdx.x / 64 takes
// the coordinates l = 4 s + q (its MFMA lane group's values), so a thread's
// stores of xr are contiguous and its loop is a quarter of the dimension.
// The centred rows and their norms come first (the median's Gram form reads
// them); X = [-(2/h) x | 1 | 0] needs h and comes after the median.
// In split form the rows are also written as three BF16 parts (thread (r, q)
// the coordinates 8 q .. 8 q + 7 of row r, as the MFMA lane group q reads
// them), which the median's Gram form and the contraction both read.  The
// spare slot 31 (d <= 31) holds e_i = -|x_i|^2 / 2's parts: as a column
// operand against (1, 0, 0) in the row operand's slot, the contraction's Gram
// adds e_j itself; the median's row operand zeroes the slot.
__device__ void pack32_x_rows(int N, int d, int ks, int row0, const float* __restrict__ theta, const View32& v,
                              bool parts) {
    __shared__ float part[4][64];
    const int r = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int i = row0 + r;
    const int kd = 4 * ks;
    float nrm = 0.0f;
    for (int s = 0; s < ks; ++s) {
        const int l = 4 * s + q;
        const float x = (i < N && l < d) ? theta[(int64_t)l * N + i] - v.ctr[l] : 0.0f;
        nrm = fmaf(x, x, nrm);
        v.xr[(int64_t)i * kd + q * ks + s] = x;
    }
    part[q][r] = nrm;
    __syncthreads();
    if (q == 0) v.nrm[i] = (part[0][r] + part[1][r]) + (part[2][r] + part[3][r]);
    __syncthreads();
    if (parts) {
        float x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int l = 8 * q + u;
            x[u] = (i < N && l < d) ? theta[(int64_t)l * N + i] - v.ctr[l] : 0.0f;
        }
        if (q == 3) x[7] = -0.5f * ((part[0][r] + part[1][r]) + (part[2][r] + part[3][r]));
        bf16x8 p0, p1, p2;
        split3(x, p0, p1, p2);
        __bf16* o = v.xs3 + (int64_t)i * 96 + 8 * q;
        *reinterpret_cast<bf16x8*>(o) = p0;
        *reinterpret_cast<bf16x8*>(o + 32) = p1;
        *reinterpret_cast<bf16x8*>(o + 64) = p2;
    }
}

// V[i][n] = w_i (g[n][i] - (2/h) x_i[n]) for n < d, w_i for n = d, 0 past it
// and for the padding rows i >= N (w_i = 1 without weights)
__device__ void pack32_v_rows(int N, int d, int ot, int row0, const float* __restrict__ theta,
                              const float* __restrict__ g, const float* __restrict__ wts, const View32& v) {
    const int r = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int i = row0 + r;
    const float c2 = 2.0f / v.sel->h;
    const float w = (i < N && wts) ? wts[i] : 1.0f;
    float* vt = v.vt + (int64_t)(i >> 4) * ot * 256 + (i & 15);
    for (int n = q; n < 16 * ot; n += 4) {
        float x = 0.0f;
        if (i < N) {
            if (n < d) x = -c2 * (theta[(int64_t)n * N + i] - v.ctr[n]) + g[(int64_t)n * N + i];
            else x = n == d ? 1.0f : 0.0f;
            if (wts) x *= w;
        }
        vt[(n >> 4) * 256 + (n & 15) * 16] = x;
    }
}

// Split form, 64 rows per 256 threads: V's parts (the rows' parts come with
// the bandwidth stage), V[i][n] as in pack32_v_rows, in the order the K.V
// product reads them: within a 32-particle chunk, column n holds 32 values
// whose slot 8 q + u is particle 4 q + (u & 3) (+ 16 for u >= 4), one 16-byte
// store per (chunk, column, q) and part.
__device__ void pack3_rows(int N, int d, int ot, int npad, int row0, const float* __restrict__ theta,
                           const float* __restrict__ g, const float* __restrict__ wts, const View32& v) {
    const int vc = 16 * ot;
    const float c2 = 2.0f / v.sel->h;
    const int64_t plane = (int64_t)npad * vc;
    for (int o = threadIdx.x; o < 8 * vc; o += 256) {  // 2 chunks x vc columns x 4 lane groups
        const int qc = (row0 >> 5) + o / (4 * vc), n = (o >> 2) % vc, q = o & 3;
        float x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = 32 * qc + 4 * q + (u & 3) + (u >= 4 ? 16 : 0);
            x[u] = 0.0f;
            if (i < N) {
                if (n < d) x[u] = -c2 * (theta[(int64_t)n * N + i] - v.ctr[n]) + g[(int64_t)n * N + i];
                else x[u] = n == d ? 1.0f : 0.0f;
                if (wts) x[u] *= wts[i];
            }
        }
        bf16x8 p0, p1, p2;
        split3(x, p0, p1, p2);
        __bf16* dst = v.vs3 + ((int64_t)qc * vc + n) * 32 + 8 * q;
        *reinterpret_cast<bf16x8*>(dst) = p0;
        *reinterpret_cast<bf16x8*>(dst + plane) = p1;
        *reinterpret_cast<bf16x8*>(dst + 2 * plane) = p2;
    }
}

// ---- contraction: partial sums of K V over the columns [j0, j1) -------------------
// V[j][n] for the lane's j = jc + 4 kq + t and n = 16 o + col, one 16-byte
// load per output tile (the tile stores the lane's four j together).
template <int OT>
__device__ __forceinline__ void load_v(int jc, int col, int kq, const View32& v, f4 (&vv)[OT]) {
    const float* vp = v.vt + (int64_t)(jc >> 4) * OT * 256 + col * 16 + kq * 4;
#pragma unroll
    for (int o = 0; o < OT; ++o) vv[o] = *reinterpret_cast<const f4*>(vp + o * 256);
}

template <int KS, int OT>
__device__ void phi32_body(int row0, int j0, int j1, int split, int npad, const View32& v) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int rbase = row0 + wave * 64;
    const float c = -1.44269504088896341f / v.sel->h;  // K = 2^(c D)
    const float m2c = -2.0f * c;
    float xi[4][KS], ni[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const float* p = v.xr + (int64_t)(rbase + 16 * r + col) * (4 * KS) + kq * KS;
#pragma unroll
        for (int s = 0; s < KS; ++s) xi[r][s] = p[s];
        ni[r] = c * v.nrm[rbase + 16 * r + col];
    }
    f4 acc[4][OT];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int o = 0; o < OT; ++o) acc[r][o] = f4{0.f, 0.f, 0.f, 0.f};
    // the next 16 columns' operands load while these compute
    float xj[KS], xn[KS];
    f4 nj, nn, vb[OT], vn[OT];
    auto load_x = [&](int jc, float (&x)[KS], f4& n) {
        const float* p = v.xr + (int64_t)(jc + col) * (4 * KS) + kq * KS;
#pragma unroll
        for (int s = 0; s < KS; ++s) x[s] = p[s];
        n = *reinterpret_cast<const f4*>(v.nrm + jc + 4 * kq);
    };
    if (j0 < j1) {
        load_x(j0, xj, nj);
        load_v<OT>(j0, col, kq, v, vb);
    }
    for (int jc = j0; jc < j1; jc += 16) {
        const bool more = jc + 16 < j1;
        if (more) {
            load_x(jc + 16, xn, nn);
            load_v<OT>(jc + 16, col, kq, v, vn);
        }
        const f4 ej = nj * -0.5f;  // e_j of the lane's four columns
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            f4 s = ej;  // x_i . x_j + e_j
#pragma unroll
            for (int k = 0; k < KS; ++k) s = __builtin_amdgcn_mfma_f32_16x16x4f32(xj[k], xi[r][k], s, 0, 0, 0);
            float kv[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) kv[t] = unit_clamp(hw_exp2(fmaf(m2c, s[t], ni[r])));
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int o = 0; o < OT; ++o)
                    acc[r][o] = __builtin_amdgcn_mfma_f32_16x16x4f32(kv[t], vb[o][t], acc[r][o], 0, 0, 0);
        }
        if (more) {
#pragma unroll
            for (int s = 0; s < KS; ++s) xj[s] = xn[s];
            nj = nn;
#pragma unroll
            for (int o = 0; o < OT; ++o) vb[o] = vn[o];
        }
    }
    float* out = v.part + (int64_t)split * (16 * OT) * npad;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int o = 0; o < OT; ++o)
            *reinterpret_cast<f4*>(out + (int64_t)(16 * o + col) * npad + rbase + 16 * r + 4 * kq) = acc[r][o];
}

// ---- split form: partial sums of K V over the columns [j0, j1) ---------------------
// Operands of one 32-column chunk as this lane holds them.
template <int OT>
struct Chunk3 {
    bf16x8 xj[3][2];  // A of the Gram, part p: row j = jc + 16 sub + l % 16 (e_j's part in slot 31)
    bf16x8 vb[3][OT]; // B of K.V, part p: V[j][16 o + l % 16], j in the permuted order
};

template <int OT>
__device__ __forceinline__ void load_x3(Chunk3<OT>& c, const View32& v, int jc, int col, int kq) {
#pragma unroll
    for (int sub = 0; sub < 2; ++sub) {
        const __bf16* x = v.xs3 + (int64_t)(jc + 16 * sub + col) * 96 + 8 * kq;
#pragma unroll
        for (int p = 0; p < 3; ++p) c.xj[p][sub] = *reinterpret_cast<const bf16x8*>(x + 32 * p);
    }
}

template <int OT>
__device__ __forceinline__ void load_v3(Chunk3<OT>& c, const View32& v, int npad, int jc, int col, int kq) {
    const int64_t plane = (int64_t)npad * 16 * OT;
    const __bf16* vch = v.vs3 + ((int64_t)(jc >> 5) * 16 * OT + col) * 32 + 8 * kq;
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int o = 0; o < OT; ++o) c.vb[p][o] = *reinterpret_cast<const bf16x8*>(vch + p * plane + 16 * o * 32);
}

// The six part products of a x b (parts 0 = hi, 1 = mid, 2 = lo) whose
// order is at least 2^-16 of it, smallest first.
__device__ constexpr int kPairs3[6][2] = {{1, 1}, {2, 0}, {0, 2}, {1, 0}, {0, 1}, {0, 0}};

// One 32-column chunk for the wave's 4 row tiles: the Gram MFMAs (x_i . x_j,
// and e_j = -|x_j|^2 / 2 from slot 31), then per row tile K = 2^(c D) split in
// three (VALU) and the K.V MFMAs.  One operand buffer: the next chunk's Gram
// operands load as soon as this chunk's Gram has read them (they arrive
// during its K.V work), its V as soon as the K.V products have read V
// (arriving during the next Gram).
template <int OT>
__device__ __forceinline__ void chunk3_step(Chunk3<OT>& cur, const bf16x8 (&xi)[3][4], const float (&ni)[4], float m2c,
                                            f4 (&acc)[4][OT], const View32& v, int npad, int jn, bool more, int col,
                                            int kq) {
    f4 s[4][2];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int sub = 0; sub < 2; ++sub) {
            s[r][sub] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int e = 0; e < 6; ++e)
                s[r][sub] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cur.xj[kPairs3[e][0]][sub], xi[kPairs3[e][1]][r],
                                                                    s[r][sub], 0, 0, 0);
        }
    if (more) load_x3<OT>(cur, v, jn, col, kq);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        float k[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) k[t] = unit_clamp(hw_exp2(fmaf(m2c, s[r][t >> 2][t & 3], ni[r])));
        bf16x8 ka[3];
        split3(k, ka[0], ka[1], ka[2]);
#pragma unroll
        for (int e = 0; e < 6; ++e)
#pragma unroll
            for (int o = 0; o < OT; ++o)
                acc[r][o] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ka[kPairs3[e][0]], cur.vb[kPairs3[e][1]][o],
                                                                    acc[r][o], 0, 0, 0);
    }
    if (more) load_v3<OT>(cur, v, npad, jn, col, kq);
}

// 64 rows from row0, columns [j0, j1) (a multiple of 128: the 4 waves take
// consecutive quarters); the waves' sums are added in wave order through LDS
// and stored as the split's partial, laid out as the FP32 form's.
template <int OT>
__device__ void phi3_body(int npad, int row0, int j0, int j1, int split, const View32& v) {
    __shared__ f4 red[3][4 * OT][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4;
    {
        const int q = (j1 - j0) >> 2;
        j0 += wave * q;
        j1 = j0 + q;
    }
    const float c = -1.44269504088896341f / v.sel->h;  // K = 2^(c D)
    const float m2c = -2.0f * c;
    bf16x8 xi[3][4];  // B of the Gram, part p, row tile r; slot 31 = (1, 0, 0) picks e_j
    float ni[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = row0 + 16 * r + col;
        const __bf16* x = v.xs3 + (int64_t)i * 96 + 8 * kq;
#pragma unroll
        for (int p = 0; p < 3; ++p) xi[p][r] = *reinterpret_cast<const bf16x8*>(x + 32 * p);
        if (kq == 3) {
            xi[0][r][7] = (__bf16)1.0f;
            xi[1][r][7] = (__bf16)0.0f;
            xi[2][r][7] = (__bf16)0.0f;
        }
        ni[r] = c * v.nrm[i];
    }
    f4 acc[4][OT];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int o = 0; o < OT; ++o) acc[r][o] = f4{0.f, 0.f, 0.f, 0.f};
    Chunk3<OT> cur;
    if (j0 < j1) {
        load_x3<OT>(cur, v, j0, col, kq);
        load_v3<OT>(cur, v, npad, j0, col, kq);
    }
    for (int jc = j0; jc < j1; jc += 32)
        chunk3_step<OT>(cur, xi, ni, m2c, acc, v, npad, jc + 32, jc + 32 < j1, col, kq);
    if (wave > 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int o = 0; o < OT; ++o) red[wave - 1][r * OT + o][lane] = acc[r][o];
    }
    __syncthreads();
    if (wave > 0) return;
#pragma unroll
    for (int u = 0; u < 3; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int o = 0; o < OT; ++o) acc[r][o] += red[u][r * OT + o][lane];
    float* out = v.part + (int64_t)split * (16 * OT) * npad;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int o = 0; o < OT; ++o)
            *reinterpret_cast<f4*>(out + (int64_t)(16 * o + col) * npad + row0 + 16 * r + 4 * kq) = acc[r][o];
}

// ---- phi from the split sums (fixed split order) ----------------------------------
// the coordinate's row and the row-sum row of every split, 16 loads in flight
// phi (stored when phi is not null) and, with upd, the operands of the
// update of Algorithm 1 on the same element (theta read for x before the
// update writes it)
__device__ ElemOut reduce32_elem(int N, int d, const SvgdLayout& L, int l, int i, const float* theta, float* phi,
                                 const View32& v, uint32_t* status, const UpdateArgs& upd, bool apply,
                                 int64_t uoff) {
    ElemOut o{true, 0.0f, uoff + (int64_t)l * N + i, {}};
    if (apply) o.in = update_load(upd, o.ue);  // issued with the sums' loads
    const int64_t sstride = (int64_t)16 * L.ot32 * L.npad;
    const float* pa = v.part + (int64_t)l * L.npad + i;
    const float* p1 = v.part + (int64_t)d * L.npad + i;
    float a = 0.0f, a1 = 0.0f;
    for (int q0 = 0; q0 < L.splits32; q0 += 8) {
        float u[8], u1[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {  // indices clamped: no load is predicated
            const int64_t o = min(q0 + k, L.splits32 - 1) * sstride;
            u[k] = pa[o];
            u1[k] = p1[o];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (q0 + k < L.splits32) {
                a += u[k];
                a1 += u1[k];
            }
    }
    const float x = theta[(int64_t)l * N + i] - v.ctr[l];
    o.r = fmaf(2.0f / v.sel->h * x, a1, a) / (float)N;
    if (phi) phi[(int64_t)l * N + i] = o.r;
    if (status && !isfinite(o.r)) atomicOr(status, STAMP_STATUS_NONFINITE_PHI);
    return o;
}

// ---- single-problem kernels -------------------------------------------------------
struct One32 {
    int N, d;
    SvgdLayout L;
};

__global__ __launch_bounds__(kMeanThreads) void k_mean(One32 a, const float* theta, char* ws) {
    particle_mean_body(a.N, blockIdx.x, theta, reinterpret_cast<float*>(ws + a.L.ctr_off));
}

__global__ __launch_bounds__(256) void k_pack32_x(One32 a, const float* theta, char* ws) {
    pack32_x_rows(a.N, a.d, a.L.ks32, blockIdx.x * 64, theta, view32(a.L, ws), a.L.split3);
}

__global__ __launch_bounds__(256) void k_pack32_v(One32 a, const float* theta, const float* g, const float* wts,
                                                  char* ws) {
    if (a.L.split3) pack3_rows(a.N, a.d, a.L.ot32, a.L.npad, blockIdx.x * 64, theta, g, wts, view32(a.L, ws));
    else pack32_v_rows(a.N, a.d, a.L.ot32, blockIdx.x * 64, theta, g, wts, view32(a.L, ws));
}

template <int KS, int OT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_phi32(One32 a, char* ws) {
    const int split = blockIdx.y;
    const int j0 = split * a.L.chunk32, j1 = min(j0 + a.L.chunk32, a.L.npad);
    phi32_body<KS, OT>(blockIdx.x * blockDim.x, j0, j1, split, a.L.npad, view32(a.L, ws));
}

// split form: 64 rows per workgroup of 256
template <int OT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_phi3(One32 a, char* ws) {
    const int split = blockIdx.y;
    const int j0 = split * a.L.chunk32, j1 = min(j0 + a.L.chunk32, a.L.npad);
    phi3_body<OT>(a.L.npad, blockIdx.x * 64, j0, j1, split, view32(a.L, ws));
}

// upd.use_adam < 0: no update
__global__ __launch_bounds__(256) void k_reduce32(One32 a, const float* theta, const float* g, float* phi, char* ws,
                                                  uint32_t* status, UpdateArgs upd) {
    __shared__ float den[2];
    const bool apply = upd.use_adam >= 0;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    ElemOut o{};
    if (e < (int64_t)a.d * a.N) {
        if (a.N == 1) o = pass_elem(g, phi, e, upd, apply);
        else o = reduce32_elem(a.N, a.d, a.L, (int)e / a.N, (int)e % a.N, theta, phi, view32(a.L, ws), status,
                               upd, apply, 0);
    }
    if (apply) {
        block_denominators(upd, den);
        if (o.ok) update_apply(upd, den, o.ue, o.in, o.r);
    }
}

// ---- batched kernels (work-list entries as in svgd.hip) ------------------------------
__device__ __forceinline__ char* base32(const ProblemDesc& D, char* ws) { return ws + D.svgd_off; }

// entry = (problem, coordinate, -, -)
// a non-null step counter is advanced once (a solve's iteration counter, read
// by the update at the iteration's end)
__global__ __launch_bounds__(kMeanThreads) void k_mean_batched(const ProblemDesc* __restrict__ descs,
                                                      const int4* __restrict__ work, const float* theta, char* ws,
                                                      int* step) {
    if (step && blockIdx.x == 0 && threadIdx.x == 0) *step += 1;
    const int4 e = work[blockIdx.x];
    const ProblemDesc& D = descs[e.x];
    particle_mean_body(D.N, e.y, theta + D.theta_off, reinterpret_cast<float*>(base32(D, ws) + D.sv.ctr_off));
}

// entry = (problem, first row of a 256-row chunk, -, -); four workgroups per
// entry, 64 rows each
__global__ __launch_bounds__(256) void k_pack32_x_batched(const ProblemDesc* __restrict__ descs,
                                                          const int4* __restrict__ work, const float* theta, char* ws) {
    const int4 e = work[blockIdx.x >> 2];
    const ProblemDesc& D = descs[e.x];
    if (D.N < 2) return;
    pack32_x_rows(D.N, D.d, D.sv.ks32, e.y + 64 * (blockIdx.x & 3), theta + D.theta_off, view32(D.sv, base32(D, ws)),
                  D.sv.split3);
}

__global__ __launch_bounds__(256) void k_pack32_v_batched(const ProblemDesc* __restrict__ descs,
                                                          const int4* __restrict__ work, const float* theta,
                                                          const float* grad, const float* wts, char* ws) {
    const int4 e = work[blockIdx.x >> 2];
    const ProblemDesc& D = descs[e.x];
    if (D.N < 2) return;
    if (D.sv.split3)
        pack3_rows(D.N, D.d, D.sv.ot32, D.sv.npad, e.y + 64 * (blockIdx.x & 3), theta + D.theta_off,
                   grad + D.theta_off, wts ? wts + D.cost_off : nullptr, view32(D.sv, base32(D, ws)));
    else
        pack32_v_rows(D.N, D.d, D.sv.ot32, e.y + 64 * (blockIdx.x & 3), theta + D.theta_off, grad + D.theta_off,
                      wts ? wts + D.cost_off : nullptr, view32(D.sv, base32(D, ws)));
}

// entry = (problem, row block of blockDim.x rows, split, -)
template <int KS, int OT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_phi32_batched(const ProblemDesc* __restrict__ descs,
                                                       const int4* __restrict__ work, char* ws) {
    const int4 e = work[blockIdx.x];
    const ProblemDesc& D = descs[e.x];
    const int j0 = e.z * D.sv.chunk32, j1 = min(j0 + D.sv.chunk32, D.sv.npad);
    phi32_body<KS, OT>(e.y * (int)blockDim.x, j0, j1, e.z, D.sv.npad, view32(D.sv, base32(D, ws)));
}

// split form: entry = (problem, 64-row block, split, -)
template <int OT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_phi3_batched(const ProblemDesc* __restrict__ descs,
                                                      const int4* __restrict__ work, char* ws) {
    const int4 e = work[blockIdx.x];
    const ProblemDesc& D = descs[e.x];
    const int j0 = e.z * D.sv.chunk32, j1 = min(j0 + D.sv.chunk32, D.sv.npad);
    phi3_body<OT>(D.sv.npad, e.y * 64, j0, j1, e.z, view32(D.sv, base32(D, ws)));
}

// entry = (problem, first element, end element, -) of the problem's d*N block
// phi may be null when the update is applied (upd.use_adam >= 0)
__global__ __launch_bounds__(256) void k_reduce32_batched(const ProblemDesc* __restrict__ descs,
                                                          const int4* __restrict__ work, const float* theta,
                                                          const float* grad, float* phi, char* ws,
                                                          uint32_t* status, UpdateArgs upd) {
    __shared__ float den[2];
    const bool apply = upd.use_adam >= 0;
    const int4 w = work[blockIdx.x];
    const ProblemDesc& D = descs[w.x];
    const int64_t e = w.y + threadIdx.x;
    ElemOut o{};
    if (e < w.z) {
        if (D.N == 1) o = pass_elem(grad, phi, D.theta_off + e, upd, apply);
        else o = reduce32_elem(D.N, D.d, D.sv, (int)e / D.N, (int)e % D.N, theta + D.theta_off,
                               phi ? phi + D.theta_off : nullptr, view32(D.sv, base32(D, ws)), status,
                               upd, apply, D.theta_off);
    }
    if (apply) {
        block_denominators(upd, den);
        if (o.ok) update_apply(upd, den, o.ue, o.in, o.r);
    }
}

// (ks, ot) of each class, in the order of phi32_class; classes 0 and 1 are
// the split form (one or two 16-column tiles of V), the rest the FP32
// matrix-core form
constexpr int kCls[kPhi32Classes][2] = {{8, 1}, {8, 2}, {8, 3}, {10, 3}, {12, 3},
                                        {12, 4}, {14, 4}, {16, 4}, {16, 5}};

template <int C>
void launch_class(dim3 grid, int rows, hipStream_t st, const One32& a, char* ws) {
    if constexpr (C < 2)
        hipLaunchKernelGGL((k_phi3<kCls[C][1]>), grid, dim3(256), 0, st, a, ws);
    else
        hipLaunchKernelGGL((k_phi32<kCls[C][0], kCls[C][1]>), grid, dim3(rows), 0, st, a, ws);
}

template <int C>
void launch_class_batched(int n, int rows, hipStream_t st, const ProblemDesc* descs, const int4* work, char* ws) {
    if constexpr (C < 2)
        hipLaunchKernelGGL((k_phi3_batched<kCls[C][1]>), dim3(n), dim3(256), 0, st, descs, work, ws);
    else
        hipLaunchKernelGGL((k_phi32_batched<kCls[C][0], kCls[C][1]>), dim3(n), dim3(rows), 0, st, descs, work, ws);
}

template <typename F>
void by_class(int c, F&& f) {
    switch (c) {
        case 0: f(std::integral_constant<int, 0>()); break;
        case 1: f(std::integral_constant<int, 1>()); break;
        case 2: f(std::integral_constant<int, 2>()); break;
        case 3: f(std::integral_constant<int, 3>()); break;
        case 4: f(std::integral_constant<int, 4>()); break;
        case 5: f(std::integral_constant<int, 5>()); break;
        case 6: f(std::integral_constant<int, 6>()); break;
        case 7: f(std::integral_constant<int, 7>()); break;
        default: f(std::integral_constant<int, 8>()); break;
    }
}

}  // namespace

int phi32_class(int d) {
    if (d <= kPhi3MaxD) return phi32_ot(d) - 1;
    const int ks = phi32_ks(d), ot = phi32_ot(d);
    for (int c = 2; c < kPhi32Classes; ++c)
        if (kCls[c][0] == ks && kCls[c][1] == ot) return c;
    return -1;
}

hipError_t launch_operands32(int N, int d, const float* theta, void* ws, const SvgdLayout& L, hipStream_t st) {
    if (N < 2) return hipSuccess;
    One32 a{N, d, L};
    char* b = static_cast<char*>(ws);
    hipLaunchKernelGGL(k_mean, dim3(d), dim3(kMeanThreads), 0, st, a, theta, b);
    hipLaunchKernelGGL(k_pack32_x, dim3(L.npad / 64), dim3(256), 0, st, a, theta, b);
    return hipGetLastError();
}

hipError_t launch_operands32_batched(const BatchPlan& P, const ProblemDesc* descs, const float* theta, char* ws,
                                     hipStream_t st, int* step) {
    if (P.n_ctr)
        hipLaunchKernelGGL(k_mean_batched, dim3(P.n_ctr), dim3(kMeanThreads), 0, st, descs, P.ctr_work, theta, ws,
                           step);
    if (P.n_row16)
        hipLaunchKernelGGL(k_pack32_x_batched, dim3(4 * P.n_row16), dim3(256), 0, st, descs, P.row16_work, theta, ws);
    return hipGetLastError();
}

hipError_t launch_svgd_direction(int N, int d, const float* theta, const float* grad_logp, float* phi, void* ws,
                                 const SvgdLayout& L, int phi_rows, uint32_t* status, hipStream_t st,
                                 const float* wts, const UpdateArgs* upd) {
    One32 a{N, d, L};
    char* b = static_cast<char*>(ws);
    if (N >= 2) {
        hipLaunchKernelGGL(k_pack32_v, dim3(L.npad / 64), dim3(256), 0, st, a, theta, grad_logp, wts, b);
        // the split form takes 64 rows per workgroup whatever the row block
        const int rows = L.split3 ? 64 : phi_rows > 0 ? phi_rows : 256;
        const dim3 grid(L.npad / rows, L.splits32);
        by_class(phi32_class(d), [&](auto c) { launch_class<decltype(c)::value>(grid, rows, st, a, b); });
    }
    const int64_t n = (int64_t)d * N;
    UpdateArgs u{};
    u.use_adam = -1;
    if (upd) u = *upd;
    hipLaunchKernelGGL(k_reduce32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, theta, grad_logp, phi, b,
                       status, u);
    return hipGetLastError();
}

hipError_t launch_svgd_direction_batched(const BatchPlan& P, const ProblemDesc* descs, const float* theta,
                                         const float* grad, float* phi, char* ws, uint32_t* status, hipStream_t st,
                                         const float* wts, const UpdateArgs* upd) {
    if (P.n_row16)
        hipLaunchKernelGGL(k_pack32_v_batched, dim3(4 * P.n_row16), dim3(256), 0, st, descs, P.row16_work, theta, grad,
                           wts, ws);
    for (int c = 0; c < kPhi32Classes; ++c)
        if (P.n_phi[c])
            by_class(c, [&](auto k) {
                launch_class_batched<decltype(k)::value>(P.n_phi[c], P.phi_rows, st, descs, P.phi_work[c], ws);
            });
    UpdateArgs u{};
    u.use_adam = -1;
    if (upd) u = *upd;
    hipLaunchKernelGGL(k_reduce32_batched, dim3(P.n_red), dim3(256), 0, st, descs, P.red_work, theta, grad, phi, ws,
                       status, u);
    return hipGetLastError();
}

}  // namespace stamp
