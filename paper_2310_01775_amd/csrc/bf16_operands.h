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

// Rows row0 .. row0 + 63 of the padded set: thread tid < 64 packs row
// row0 + tid (the other threads return).  Padding rows (i >= N) hold x^ = 0
// and e = 0, so every kernel value with them stays finite (and their V rows
// are zero).  kd >= d + 2.
__device__ __forceinline__ void pack16_theta_rows(int N, int d, int kd, int row0, int tid,
                                                  const float* __restrict__ theta, const float* __restrict__ ctr,
                                                  float scale, __bf16* __restrict__ xr, __bf16* __restrict__ xc,
                                                  float* __restrict__ nrm) {
    typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
    if (tid >= 64) return;
    const int i = row0 + tid;
    auto coord = [&](int l) -> __bf16 {
        return (__bf16)((i < N && l < d) ? scale * (theta[(int64_t)l * N + i] - ctr[l]) : 0.0f);
    };
    float n = 0.0f;
    for (int l = 0; l < d; ++l) {
        const float x = (float)coord(l);
        n = fmaf(x, x, n);
    }
    const float e = -0.5f * n;
    const __bf16 hi = (__bf16)e, lo = (__bf16)(e - (float)hi);
    const __bf16 one = (__bf16)1.0f;
    for (int l0 = 0; l0 < kd; l0 += 8) {
        bf16x8_t a, c;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int l = l0 + k;
            const __bf16 x = coord(l);
            a[k] = l == d ? hi : l == d + 1 ? lo : x;
            c[k] = (l == d || l == d + 1) ? one : x;
        }
        *reinterpret_cast<bf16x8_t*>(xr + (int64_t)i * kd + l0) = a;
        *reinterpret_cast<bf16x8_t*>(xc + (int64_t)i * kd + l0) = c;
    }
    nrm[i] = e;
}

}  // namespace stamp
