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

// Same transform on sequences spaced `ss` complex values apart, with two radix-2 stages
// per pass: each thread takes the quartet (a, a + h, a + 2h, a + 3h) of stages h and 2h
// through registers, so every value makes half as many LDS round trips and the block
// half as many barriers.  The butterflies, their twiddles and their order are those of
// the radix-2 transform above.  Neighbouring threads work on neighbouring sequences: with
// ss = n + 1 (odd) their accesses fall in distinct LDS banks at every stage.
__device__ inline void bfly(double2& x, double2& y, double2 w) {
    const double2 t = cmul(y, w);
    y = make_double2(x.x - t.x, x.y - t.y);
    x = make_double2(x.x + t.x, x.y + t.y);
}

template <bool INV>
__device__ inline double2 twid(const double2* __restrict__ tw, int i) {
    double2 w = tw[i];
    if (INV) w.y = -w.y;
    return w;
}

template <bool INV>
__device__ inline void lds_fft_s(double2* s, int nb, int ss, int logn, const double2* __restrict__ tw) {
    const int n = 1 << logn;
    int lh = 0;
    if (logn & 1) {                              // odd length exponent: one single stage first
        const int hn = n >> 1;
        for (int t = threadIdx.x; t < nb * hn; t += blockDim.x) {
            const int seq = t % nb, bf = t / nb;
            const int a = seq * ss + 2 * bf;
            double2 x = s[a], y = s[a + 1];
            bfly(x, y, twid<INV>(tw, 0));
            s[a] = x;
            s[a + 1] = y;
        }
        __syncthreads();
        lh = 1;
    }
    for (; lh < logn; lh += 2) {
        const int h = 1 << lh;
        const int nq = n >> 2;                   // quartets per sequence
        const int t1 = logn - 1 - lh, t2 = logn - 2 - lh;
        for (int t = threadIdx.x; t < nb * nq; t += blockDim.x) {
            const int seq = t % nb, qd = t / nb;
            const int j = qd & (h - 1), grp = qd >> lh;
            const int a = seq * ss + (grp << (lh + 2)) + j;
            double2 x0 = s[a], x1 = s[a + h], x2 = s[a + 2 * h], x3 = s[a + 3 * h];
            const double2 w1 = twid<INV>(tw, j << t1);
            bfly(x0, x1, w1);
            bfly(x2, x3, w1);
            bfly(x0, x2, twid<INV>(tw, j << t2));
            bfly(x1, x3, twid<INV>(tw, (j + h) << t2));
            s[a] = x0;
            s[a + h] = x1;
            s[a + 2 * h] = x2;
            s[a + 3 * h] = x3;
        }
        __syncthreads();
    }
}

// Decimation in frequency on the same layout: natural-order input, bit-reversed output
// (s[p] = X(bitrev p)), stages of half length n/2, n/4, ..., 2^stop (the stages below
// 2^stop are left to the caller, who runs them in registers on four consecutive values).
// A butterfly (x, y) -> (x + y, (x - y) w), w = tw[j n / (2 half)] (conjugate for the
// inverse).  With an odd stage count the first stage runs alone, then pairs (2h, h) on
// quartets, neighbouring threads on neighbouring sequences.
__device__ inline void dif(double2& x, double2& y, double2 w) {
    const double2 d = make_double2(x.x - y.x, x.y - y.y);
    x = make_double2(x.x + y.x, x.y + y.y);
    y = cmul(d, w);
}

template <bool INV>
__device__ inline void lds_fft_dif_s(double2* s, int nb, int ss, int logn, int stop,
                                     const double2* __restrict__ tw) {
    const int n = 1 << logn;
    int lh = logn - 1;                            // log2 of the current half length
    if ((logn - stop) & 1) {
        const int half = 1 << lh;                 // = n / 2, twiddle index j
        for (int t = threadIdx.x; t < nb * half; t += blockDim.x) {
            const int seq = t % nb, j = t / nb;
            const int a = seq * ss + j;
            double2 x = s[a], y = s[a + half];
            dif(x, y, twid<INV>(tw, j));
            s[a] = x;
            s[a + half] = y;
        }
        __syncthreads();
        --lh;
    }
    for (; lh > stop; lh -= 2) {                  // stages 2h = 2^lh and h = 2^(lh-1)
        const int h = 1 << (lh - 1);
        const int nq = n >> 2;
        const int sa = logn - 1 - lh;             // twiddle stride of the 2h stage: n / (4h)
        for (int t = threadIdx.x; t < nb * nq; t += blockDim.x) {
            const int seq = t % nb, qd = t / nb;
            const int j = qd & (h - 1), grp = qd >> (lh - 1);
            const int a = seq * ss + (grp << (lh + 1)) + j;
            double2 x0 = s[a], x1 = s[a + h], x2 = s[a + 2 * h], x3 = s[a + 3 * h];
            dif(x0, x2, twid<INV>(tw, j << sa));
            dif(x1, x3, twid<INV>(tw, (j + h) << sa));
            const double2 wc = twid<INV>(tw, j << (sa + 1));
            dif(x0, x1, wc);
            dif(x2, x3, wc);
            s[a] = x0;
            s[a + h] = x1;
            s[a + 2 * h] = x2;
            s[a + 3 * h] = x3;
        }
        __syncthreads();
    }
}
