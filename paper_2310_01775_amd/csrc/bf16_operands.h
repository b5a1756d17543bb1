// Theta operands of the BF16 matrix-core form of the SVGD direction, shared by
// the contraction's file and the fused bandwidth-stage kernels of the
// sampled median: the centred rows x~_i = bf16(theta_i - c) and
// e_i = -|x~_i|^2 / 2 (the Gram accumulator's starting value), with c the
// particle mean (Sec. III-C's RBF kernel depends on differences only, so the
// centre changes nothing but rounding; it keeps x~ small).
#pragma once

#include "common.h"

namespace stamp {

// Threads of the BF16 form's centre (one workgroup per coordinate).
constexpr int kCentreThreads = 256;

// Rows row0 .. row0 + 63 of the padded set, by 256 threads (tid): a thread
// per (row, group of 8 coordinates) makes one 16-byte store; the groups of a
// row sit in adjacent lanes and add their norms by exchange.  kd = 32 or 64.
__device__ __forceinline__ void pack16_theta_rows(int N, int d, int kd, int row0, int tid,
                                                  const float* __restrict__ theta, const float* __restrict__ ctr,
                                                  __bf16* __restrict__ xb, float* __restrict__ nrm) {
    typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
    const int groups = kd >> 3;  // 4 or 8: every thread takes the same number of steps
    for (int o = tid; o < 64 * groups; o += 256) {
        const int i = row0 + o / groups, l0 = 8 * (o & (groups - 1));
        bf16x8_t x8;
        float n = 0.0f;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int l = l0 + k;
            float x = 0.0f;
            if (i < N && l < d) x = theta[(int64_t)l * N + i] - ctr[l];
            x8[k] = (__bf16)x;
            const float xr = (float)x8[k];
            n = fmaf(xr, xr, n);
        }
        *reinterpret_cast<bf16x8_t*>(xb + (int64_t)i * kd + l0) = x8;
        for (int m = 1; m < groups; m <<= 1) n += __shfl_xor(n, m);
        if (l0 == 0) nrm[i] = -0.5f * n;
    }
}

}  // namespace stamp
