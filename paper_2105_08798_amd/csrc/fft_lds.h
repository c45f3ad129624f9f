// Batched radix-2 FFT on sequences held in LDS (gfx950).
//
// nb sequences of length n = 2^logn are stored back to back in `s` (double2 = complex),
// already permuted to bit-reversed order by the loader.  Decimation in time, one
// __syncthreads per stage.  tw[j] = exp(-2 pi i j / n), j < n/2, comes from a table the
// host computed in extended precision; the inverse transform uses conjugate twiddles
// and no scaling.  Every thread of the block must call this function.
#pragma once
#include <hip/hip_runtime.h>

__device__ inline unsigned bitrev(unsigned x, int logn) {
    return logn ? (__brev(x) >> (32 - logn)) : 0u;
}

__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ inline void lds_fft(double2* s, int nb, int logn, const double2* __restrict__ tw,
                               bool inverse) {
    const int n = 1 << logn;
    const int hn = n >> 1;
    const int total = nb * hn;
    for (int lh = 0; lh < logn; ++lh) {          // half = 2^lh, len = 2^(lh+1)
        const int half = 1 << lh;
        const int tws = logn - 1 - lh;           // twiddle stride log2(n / len)
        for (int t = threadIdx.x; t < total; t += blockDim.x) {
            const int seq = t >> (logn - 1);
            const int bf = t & (hn - 1);
            const int j = bf & (half - 1);
            const int grp = bf >> lh;
            const int a = seq * n + (grp << (lh + 1)) + j;
            const int b = a + half;
            double2 w = tw[j << tws];
            if (inverse) w.y = -w.y;
            const double2 x = s[a];
            const double2 y = cmul(s[b], w);
            s[a] = make_double2(x.x + y.x, x.y + y.y);
            s[b] = make_double2(x.x - y.x, x.y - y.y);
        }
        __syncthreads();
    }
}
