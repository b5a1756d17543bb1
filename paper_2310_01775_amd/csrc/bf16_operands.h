// Theta operands of the BF16 matrix-core form of the SVGD direction: the
// scaled centred rows x^_i = bf16(sqrt(m) (theta_i - c)), with c the particle
// mean (Sec. III-C's RBF kernel depends on differences only, so the centre
// changes nothing but rounding; it keeps x^ small) and m = 2 log2(e) / h, so
// that log2 K_ij = -(m / 2) |x_i - x_j|^2 = x^_i . x^_j + e_i + e_j with
// e_i = -|x^_i|^2 / 2 (in FP32, from the rounded rows, so that the distance
// of a row to itself is zero but for the accumulation's rounding).  The row
// operand carries e_i in two more Gram columns as a BF16 pair (hi, lo =
// bf16(e_i - hi); their sum is e_i to within 2^-18 |e_i|), the column operand
// carries 1 in both, and e_j is the Gram accumulator's starting value: the
// Gram MFMA then gives log2 K_ij itself.
#pragma once

#include "common.h"

namespace stamp {

// Threads of the BF16 form's centre (one workgroup per coordinate).
constexpr int kCentreThreads = 256;

// Rows row0 .. row0 + 63 of the padded set, by the 256 threads of a
// workgroup (tid; every thread must call it, it holds a barrier): a thread per
// (group of 8 coordinates, row), rows fastest so the loads of a coordinate
// are contiguous; the groups' partial norms meet in LDS and every row adds
// its own in group order.  Padding rows (i >= N) hold x^ = 0 and e = 0, so
// every kernel value with them stays finite (and their V rows are zero).
// kd >= d + 2, kd <= 96.
__device__ __forceinline__ void pack16_theta_rows(int N, int d, int kd, int row0, int tid,
                                                  const float* __restrict__ theta, const float* __restrict__ ctr,
                                                  float scale, __bf16* __restrict__ xr, __bf16* __restrict__ xc,
                                                  float* __restrict__ nrm) {
    typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
    constexpr int kSteps = 3;  // 64 rows x 12 groups at kd = 96, over 256 threads
    __shared__ float part[12][64];
    const int groups = kd >> 3;
    bf16x8_t x8[kSteps];
#pragma unroll
    for (int k = 0; k < kSteps; ++k) {
        const int o = tid + 256 * k, r = o & 63, g = o >> 6, i = row0 + r;
        if (g < groups) {
            float n = 0.0f;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int l = 8 * g + u;
                x8[k][u] = (__bf16)((i < N && l < d) ? scale * (theta[(int64_t)l * N + i] - ctr[l]) : 0.0f);
                const float x = (float)x8[k][u];
                n = fmaf(x, x, n);
            }
            part[g][r] = n;
        }
    }
    __syncthreads();
    const __bf16 one = (__bf16)1.0f;
#pragma unroll
    for (int k = 0; k < kSteps; ++k) {
        const int o = tid + 256 * k, r = o & 63, g = o >> 6, i = row0 + r;
        if (g < groups) {
            float n = 0.0f;
            for (int q = 0; q < groups; ++q) n += part[q][r];
            const float e = -0.5f * n;
            const __bf16 hi = (__bf16)e, lo = (__bf16)(e - (float)hi);
            bf16x8_t a = x8[k], c = x8[k];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int l = 8 * g + u;
                if (l == d) a[u] = hi;
                if (l == d + 1) a[u] = lo;
                if (l == d || l == d + 1) c[u] = one;
            }
            *reinterpret_cast<bf16x8_t*>(xr + (int64_t)i * kd + 8 * g) = a;
            *reinterpret_cast<bf16x8_t*>(xc + (int64_t)i * kd + 8 * g) = c;
            if (g == 0) nrm[i] = e;
        }
    }
}

}  // namespace stamp
