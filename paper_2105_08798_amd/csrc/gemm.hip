// Per-mode complex products w^(m) = G^(m) f^(m) on MFMA (Section 2.3.2,
// eq. flexbc.up=Gpipl*fipl; Section 3.2, eq. impl.up=Gpipl*fipl_mvm, one dense product
// per line mode).  The complex product is one real product: A[row][k'] holds
// (Re, Im) of G^ interleaved along k', and the B operand holds, per RHS, the two
// columns (Re f, -Im f) and (Im f, Re f), so a 16-column output tile carries the real
// parts of 8 RHS in columns 0..7 and their imaginary parts in columns 8..15.
//
// A is streamed once from HBM in MFMA fragment order (each wave-wide 16-byte load is
// 1 KiB contiguous, no LDS) from the compact store: a job's stored blocks are the K
// chunks of its (mode, row tile) window, one contiguous run, K-major across the tile's
// row blocks, so a work group streams one sequential region; B fragments are re-read by
// every row tile of the same mode and stay in L2 because the job list gives all tiles
// of a mode to one XCD.
// Each work group is 4 waves; a wave owns RB row blocks (16 rows each) of one mode and
// all column tiles of that mode, over the whole K.  Loads run PF steps ahead.
#include <cstdint>

#include "kernels.h"

#include <algorithm>
#include <map>
#include <mutex>

static __device__ inline void store_c_f64(double* __restrict__ c, const GemmJob& jb, int rb,
                                          int ctile, int lane, const d4_t& acc) {
    const int64_t mp = (int64_t)jb.mb * 16;
    const int col = lane & 15;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int row = 16 * rb + 4 * j + (lane >> 4);      // FP64 16x16x4 output order
        c[jb.c_off + ((int64_t)ctile * mp + row) * jb.crs + col] = acc[j];
    }
}
static __device__ inline void store_c_f32acc(double* __restrict__ c, const GemmJob& jb, int rb,
                                             int ctile, int lane, const d4_t& acc) {
    const int64_t mp = (int64_t)jb.mb * 16;
    const int col = lane & 15;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int row = 16 * rb + 4 * (lane >> 4) + j;      // FP32-accumulator output order
        c[jb.c_off + ((int64_t)ctile * mp + row) * jb.crs + col] = acc[j];
    }
}

// Loads of the stored G^ blocks: every byte is read once per update, so they go out as
// nontemporal (streaming) loads and do not push the f^ fragments, the partial outputs and
// the caller's arrays out of L2 and the Infinity Cache (measured on MI355X: the products
// run 8-11 % faster than with ordinary loads).
__device__ inline double2 ld_stream(const double2* p) {
    typedef double dv2_t __attribute__((ext_vector_type(2)));
    const dv2_t v = __builtin_nontemporal_load((const dv2_t*)p);
    return make_double2(v[0], v[1]);
}
__device__ inline float4 ld_stream(const float4* p) {
    const f4_t v = __builtin_nontemporal_load((const f4_t*)p);
    return make_float4(v[0], v[1], v[2], v[3]);
}
__device__ inline bf8_t ld_stream(const bf8_t* p) { return __builtin_nontemporal_load(p); }
__device__ inline h8_t ld_stream(const h8_t* p) { return __builtin_nontemporal_load(p); }

// Persistent work-queue form of the product kernels: as many work groups as fit on the
// chip at once, each taking the next job of its list from a device counter until the
// lists are exhausted (with a list longest first, the groups that finish early take the
// short jobs: dynamic longest-processing-time scheduling of uneven jobs).  With one list
// per XCD (PqLists), the groups of an XCD work through consecutive row tiles of the same
// mode together, so the f^ fragments of their overlapping K windows are fetched into that
// XCD's L2 once; a group whose list is exhausted takes jobs from the other lists in turn.
// The last group to leave sets the counters back to zero for the next launch (so the
// launch can be replayed from a graph).  `cur` (thread 0's) counts the lists this group
// has exhausted; every group leaves once it has drawn past the end of all of them.
__device__ inline int pq_next(const PqLists& q, int* slot, int& cur) {
    if (threadIdx.x == 0) {
        const int home = q.nl > 1 ? (int)(blockIdx.x % q.nl) : 0;
        int j = 0x7fffffff;
        while (cur < q.nl) {
            const int l = (home + cur) % q.nl;
            const int s = atomicAdd(&q.ctr[l], 1);
            if (s < q.start[l + 1] - q.start[l]) {
                j = q.start[l] + s;
                break;
            }
            ++cur;
        }
        *slot = j;
    }
    __syncthreads();
    const int j = __builtin_amdgcn_readfirstlane(*slot);   // uniform: the job fields go to SGPRs
    __syncthreads();                     // every thread has read the slot; LDS of the last job free
    return j;
}
__device__ inline void pq_done(const PqLists& q) {
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&q.ctr[8], 1) == (int)gridDim.x - 1) {
            for (int l = 0; l < q.nl; ++l) atomicExch(&q.ctr[l], 0);
            atomicExch(&q.ctr[8], 0);
        }
    }
}

// Work groups of a persistent launch: the kernel's occupancy per CU times the CUs
// (queried once per kernel and cached; the library runs on one device type per process).
template <typename K>
static int pq_groups_of(K kernel, int threads) {
    static std::mutex mu;
    static std::map<const void*, int> cache;
    std::lock_guard<std::mutex> lock(mu);
    const void* key = (const void*)kernel;
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int per_cu = 0, dev = 0, cus = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0);
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int g = std::max(1, per_cu) * std::max(1, cus);
    cache[key] = g;
    return g;
}

// ------------------------------- FP64 ---------------------------------------------
// Branch-free main loop: the planner pads rows to whole work-group tiles (zero rows),
// K' to a multiple of 64 and gives every cell of a context the same column-tile count,
// so every wave runs full RB x CT tiles over the whole K; the prefetch index is clamped
// to the last step instead of being predicated.
template <int RB, int CT, int PF>
__device__ inline void gemm_f64_job(const GemmJob& jb,
                                                  const double* __restrict__ A,
                                                  const double* __restrict__ B,
                                                  double* __restrict__ C) {
    // the main loop runs whole ring passes: the ring must divide the 8 steps of a 64-k' chunk
    static_assert(8 % PF == 0, "ring depth must divide the steps of a chunk");
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rbw = jb.rb0 + wave * RB;
    if (rbw >= jb.mb) return;
    const int kp8 = jb.kp >> 3;
    const int pb = jb.k0 >> 3, pe = jb.k1 >> 3;
    constexpr int TRB = 4 * RB;          // row blocks of the tile: the A step stride
    const double2* a = (const double2*)(A + jb.a_off) + (int64_t)(wave * RB) * 64 + lane;
    const double2* b = (const double2*)(B + jb.b_off) + bpos(lane);
    d4_t acc[RB][CT];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[r][c] = (d4_t){0, 0, 0, 0};
    if (pe <= pb) {              // empty K slice: its partial output is zero
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int c = 0; c < CT; ++c) store_c_f64(C, jb, rbw + r, c, lane, acc[r][c]);
        return;
    }
    double2 ab[PF][RB], bb[PF][CT];
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        const int pw = wrap_k(pb + u, kp8);
        const int pa = min(u, pe - pb - 1);       // A: step inside the job's stored run
#pragma unroll
        for (int r = 0; r < RB; ++r) ab[u][r] = ld_stream(a + (((int64_t)pa * TRB + r) * 64));
#pragma unroll
        for (int c = 0; c < CT; ++c) bb[u][c] = b[((int64_t)c * kp8 + pw) * 64];

        // keeps the ring's loads in slot order (slot 0 first), so the first wait of the main
        // loop leaves the later slots in flight instead of draining every load
        __builtin_amdgcn_sched_barrier(0);
    }
    for (int p0 = pb; p0 < pe; p0 += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int r = 0; r < RB; ++r)
#pragma unroll
                    for (int c = 0; c < CT; ++c)
                        acc[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                            h ? ab[u][r].y : ab[u][r].x, h ? bb[u][c].y : bb[u][c].x, acc[r][c], 0, 0, 0);
            const int pl = min(p0 + u + PF, pe - 1);
            const int pn = wrap_k(pl, kp8);
#pragma unroll
            for (int r = 0; r < RB; ++r) ab[u][r] = ld_stream(a + (((int64_t)(pl - pb) * TRB + r) * 64));
#pragma unroll
            for (int c = 0; c < CT; ++c) bb[u][c] = b[((int64_t)c * kp8 + pn) * 64];
        }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < CT; ++c) store_c_f64(C, jb, rbw + r, c, lane, acc[r][c]);
}

template <int RB, int CT, int PF>
__global__ void __launch_bounds__(256) k_gemm_f64(const GemmJob* __restrict__ jobs, const double* __restrict__ A,
        const double* __restrict__ B, double* __restrict__ C) {
    const GemmJob jb = jobs[blockIdx.x];
    gemm_f64_job<RB, CT, PF>(jb, A, B, C);
}
template <int RB, int CT, int PF>
__global__ void __launch_bounds__(256) k_gemm_f64_pq(const GemmJob* __restrict__ jobs, int njobs, PqLists q,
        const double* __restrict__ A, const double* __restrict__ B, double* __restrict__ C) {
    __shared__ int slot;
    int cur = 0;
    for (int j = pq_next(q, &slot, cur); j < njobs; j = pq_next(q, &slot, cur)) {
        const GemmJob jb = jobs[j];
        gemm_f64_job<RB, CT, PF>(jb, A, B, C);
    }
    pq_done(q);
}

// ------------------------------- FP32 ---------------------------------------------
// FP32 MFMA with FP32 accumulation inside chunks of KCH*16 real k, FP64 across chunks.
template <int RB, int CT, int PF, int KCH>
__device__ inline void gemm_f32_job(const GemmJob& jb,
                                                  const float* __restrict__ A,
                                                  const float* __restrict__ B,
                                                  double* __restrict__ C) {
    static_assert(4 % PF == 0, "ring depth must divide the 4 steps of a 64-k' chunk");
    static_assert(KCH % PF == 0, "FP32 chunks are whole ring passes");
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rbw = jb.rb0 + wave * RB;
    if (rbw >= jb.mb) return;
    const int kq = jb.kp >> 4;
    const int qb = jb.k0 >> 4, qe = jb.k1 >> 4;
    constexpr int TRB = 4 * RB;          // row blocks of the tile: the A step stride
    const float4* a = (const float4*)(A + jb.a_off) + (int64_t)(wave * RB) * 64 + lane;
    const float4* b = (const float4*)(B + jb.b_off) + bpos(lane);
    d4_t acc[RB][CT];
    f4_t ac32[RB][CT];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            acc[r][c] = (d4_t){0, 0, 0, 0};
            ac32[r][c] = (f4_t){0, 0, 0, 0};
        }
    if (qe <= qb) {              // empty K slice: its partial output is zero
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int c = 0; c < CT; ++c) store_c_f32acc(C, jb, rbw + r, c, lane, acc[r][c]);
        return;
    }
    float4 ab[PF][RB], bb[PF][CT];
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        const int qw = wrap_k(qb + u, kq);
        const int qa = min(u, qe - qb - 1);       // A: step inside the job's stored run
#pragma unroll
        for (int r = 0; r < RB; ++r) ab[u][r] = ld_stream(a + (((int64_t)qa * TRB + r) * 64));
#pragma unroll
        for (int c = 0; c < CT; ++c) bb[u][c] = b[((int64_t)c * kq + qw) * 64];

        // keeps the ring's loads in slot order (slot 0 first), so the first wait of the main
        // loop leaves the later slots in flight instead of draining every load
        __builtin_amdgcn_sched_barrier(0);
    }
    for (int q0 = qb; q0 < qe; q0 += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
#pragma unroll
            for (int h = 0; h < 4; ++h)
#pragma unroll
                for (int r = 0; r < RB; ++r)
#pragma unroll
                    for (int c = 0; c < CT; ++c) {
                        const float av = h == 0 ? ab[u][r].x : h == 1 ? ab[u][r].y : h == 2 ? ab[u][r].z : ab[u][r].w;
                        const float bv = h == 0 ? bb[u][c].x : h == 1 ? bb[u][c].y : h == 2 ? bb[u][c].z : bb[u][c].w;
                        ac32[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, ac32[r][c], 0, 0, 0);
                    }
            const int ql = min(q0 + u + PF, qe - 1);
            const int qn = wrap_k(ql, kq);
#pragma unroll
            for (int r = 0; r < RB; ++r) ab[u][r] = ld_stream(a + (((int64_t)(ql - qb) * TRB + r) * 64));
#pragma unroll
            for (int c = 0; c < CT; ++c) bb[u][c] = b[((int64_t)c * kq + qn) * 64];

            __builtin_amdgcn_sched_barrier(0);     // the same order in every ring pass
        }
        if (((q0 - qb + PF) % KCH) == 0 || q0 + PF >= qe) {
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int c = 0; c < CT; ++c) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[r][c][j] += (double)ac32[r][c][j];
                    ac32[r][c] = (f4_t){0, 0, 0, 0};
                }
        }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < CT; ++c) store_c_f32acc(C, jb, rbw + r, c, lane, acc[r][c]);
}

template <int RB, int CT, int PF, int KCH>
__global__ void __launch_bounds__(256) k_gemm_f32(const GemmJob* __restrict__ jobs, const float* __restrict__ A,
        const float* __restrict__ B, double* __restrict__ C) {
    const GemmJob jb = jobs[blockIdx.x];
    gemm_f32_job<RB, CT, PF, KCH>(jb, A, B, C);
}
template <int RB, int CT, int PF, int KCH>
__global__ void __launch_bounds__(256) k_gemm_f32_pq(const GemmJob* __restrict__ jobs, int njobs, PqLists q,
        const float* __restrict__ A, const float* __restrict__ B, double* __restrict__ C) {
    __shared__ int slot;
    int cur = 0;
    for (int j = pq_next(q, &slot, cur); j < njobs; j = pq_next(q, &slot, cur)) {
        const GemmJob jb = jobs[j];
        gemm_f32_job<RB, CT, PF, KCH>(jb, A, B, C);
    }
    pq_done(q);
}

// ------------------------------- split BF16 ---------------------------------------
// G ~ G_hi + G_lo, f ~ f_hi + f_lo; products lo*hi + hi*lo + hi*hi on BF16 MFMA with
// FP32 accumulation inside chunks of KCH*32 real k, FP64 across chunks.
// The split-FP16 form runs the same kernel on FP16 MFMA; its operands carry power-of-two
// scales that the inverse transform removes.
__device__ inline f4_t mfma_16x16x32(bf8_t a, bf8_t b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ inline f4_t mfma_16x16x32(h8_t a, h8_t b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

template <typename VT, int RB, int CT, int PF, int KCH>
__device__ inline void gemm_split_job(const GemmJob& jb,
                                                    const unsigned short* __restrict__ A,
                                                    const unsigned short* __restrict__ B,
                                                    double* __restrict__ C) {
    static_assert(2 % PF == 0, "ring depth must divide the 2 steps of a 64-k' chunk");
    static_assert(KCH % PF == 0, "FP32 chunks are whole ring passes");
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rbw = jb.rb0 + wave * RB;
    if (rbw >= jb.mb) return;
    const int kt = jb.kp >> 5;
    const int tb = jb.k0 >> 5, te = jb.k1 >> 5;
    // 16-byte units: per (block, t): hi run of 64 units then lo run of 64 units
    constexpr int TRB = 4 * RB;          // row blocks of the tile: the A step stride
    const VT* a = (const VT*)(A + jb.a_off) + (int64_t)(wave * RB) * 128 + lane;
    const VT* b = (const VT*)(B + jb.b_off) + bpos(lane);
    d4_t acc[RB][CT];
    f4_t ac32[RB][CT];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            acc[r][c] = (d4_t){0, 0, 0, 0};
            ac32[r][c] = (f4_t){0, 0, 0, 0};
        }
    if (te <= tb) {              // empty K slice: its partial output is zero
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int c = 0; c < CT; ++c) store_c_f32acc(C, jb, rbw + r, c, lane, acc[r][c]);
        return;
    }
    VT ah[PF][RB], al[PF][RB], bh[PF][CT], bl[PF][CT];
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        const int tw = wrap_k(tb + u, kt);
        const int ta = min(u, te - tb - 1);       // A: step inside the job's stored run
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            ah[u][r] = ld_stream(a + (((int64_t)ta * TRB + r) * 128));
            al[u][r] = ld_stream(a + (((int64_t)ta * TRB + r) * 128 + 64));
        }
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            bh[u][c] = b[((int64_t)c * kt + tw) * 128];
            bl[u][c] = b[((int64_t)c * kt + tw) * 128 + 64];
        }
        // keeps the ring's loads in slot order (slot 0 first), so the first wait of the main
        // loop leaves the later slots in flight instead of draining every load
        __builtin_amdgcn_sched_barrier(0);
    }
    for (int t0 = tb; t0 < te; t0 += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int c = 0; c < CT; ++c)
                    ac32[r][c] = mfma_16x16x32(al[u][r], bh[u][c], ac32[r][c]);
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int c = 0; c < CT; ++c)
                    ac32[r][c] = mfma_16x16x32(ah[u][r], bl[u][c], ac32[r][c]);
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int c = 0; c < CT; ++c)
                    ac32[r][c] = mfma_16x16x32(ah[u][r], bh[u][c], ac32[r][c]);
            const int tl = min(t0 + u + PF, te - 1);
            const int tn = wrap_k(tl, kt);
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                ah[u][r] = ld_stream(a + (((int64_t)(tl - tb) * TRB + r) * 128));
                al[u][r] = ld_stream(a + (((int64_t)(tl - tb) * TRB + r) * 128 + 64));
            }
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                bh[u][c] = b[((int64_t)c * kt + tn) * 128];
                bl[u][c] = b[((int64_t)c * kt + tn) * 128 + 64];
            }
            __builtin_amdgcn_sched_barrier(0);     // the same order in every ring pass
        }
        if (((t0 - tb + PF) % KCH) == 0 || t0 + PF >= te) {
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int c = 0; c < CT; ++c) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[r][c][j] += (double)ac32[r][c][j];
                    ac32[r][c] = (f4_t){0, 0, 0, 0};
                }
        }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < CT; ++c) store_c_f32acc(C, jb, rbw + r, c, lane, acc[r][c]);
}

template <typename VT, int RB, int CT, int PF, int KCH>
__global__ void __launch_bounds__(256) k_gemm_split(const GemmJob* __restrict__ jobs, const unsigned short* __restrict__ A,
        const unsigned short* __restrict__ B, double* __restrict__ C) {
    const GemmJob jb = jobs[blockIdx.x];
    gemm_split_job<VT, RB, CT, PF, KCH>(jb, A, B, C);
}
template <typename VT, int RB, int CT, int PF, int KCH>
__global__ void __launch_bounds__(256) k_gemm_split_pq(const GemmJob* __restrict__ jobs, int njobs, PqLists q,
        const unsigned short* __restrict__ A, const unsigned short* __restrict__ B, double* __restrict__ C) {
    __shared__ int slot;
    int cur = 0;
    for (int j = pq_next(q, &slot, cur); j < njobs; j = pq_next(q, &slot, cur)) {
        const GemmJob jb = jobs[j];
        gemm_split_job<VT, RB, CT, PF, KCH>(jb, A, B, C);
    }
    pq_done(q);
}

// Variant for 4 or 8 column tiles (many RHS): the B fragments of a K step are the same
// for the NW waves of a work group, so they are loaded once per work group into LDS
// (double buffered) instead of once per wave from L2, and the group meets at one barrier
// per S steps.  NW waves per group: four at 64 RHS (the FP64 accumulators of 16 output
// tiles and the A and B rings need more registers than two waves per SIMD leave, so a
// group of eight waves, which would halve the B fetches per row, spills).  A is streamed from HBM into a register ring PFA steps deep.  Each thread
// also keeps its share of B for the same PFA steps in a ring of its own: vector-memory
// loads complete in issue order, so the wait for B before it is copied into LDS would
// otherwise also wait for every A load issued before it, and cut the effective depth of
// the A ring down to the distance at which B was fetched.  K windows and slices hold an
// even number of steps, so S = 2 needs no tail.
// CH = 2 splits the column tiles between two halves of the waves (eight waves: four row
// groups x two column halves, the same 128-row tile): each wave holds the accumulators of
// half the tiles, so two waves fit per SIMD; the two waves of a row group read the same A
// (ordinary loads, so the second finds it in L2).  Every output tile sees the same
// sequence of MFMAs, so the result is bitwise that of CH = 1.
template <typename VT, int RB, int CT, int PFA, int KCH, int S, int NW, int CH = 1>
__device__ inline void gemm_split_lds_job(const GemmJob& jb,
                                                        const unsigned short* __restrict__ A,
                                                        const unsigned short* __restrict__ B,
                                                        double* __restrict__ C) {
    static_assert(CT >= 2 && (CT % 2) == 0, "B staging assumes an even tile count");
    static_assert(CH == 1 || CH == 2, "one or two column halves");
    static_assert(NW % CH == 0 && ((CT / CH) % 2) == 0, "column halves of an even tile count");
    static_assert(S == 1 || S == 2, "one or two K steps per barrier");
    constexpr int RG = NW / CH;              // row groups of the tile
    constexpr int CTW = CT / CH;             // column tiles per wave
    static_assert(PFA >= 2 * S && (PFA % (2 * S)) == 0, "ring depth must be a multiple of 2 S");
    constexpr int NTH = 64 * NW;             // threads of the work group
    constexpr int STEP_UNITS = CT * 128;     // 16-byte units of B per step (hi and lo runs)
    static_assert(STEP_UNITS % NTH == 0, "B units must spread evenly over the threads");
    constexpr int NU = STEP_UNITS / NTH;     // per thread and step
    __shared__ VT bs[2][STEP_UNITS * S];
    if (jb.rb0 >= jb.mb) return;             // whole work group (empty job)
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int rg = wave % RG, c0w = (wave / RG) * CTW;
    const int rbw = jb.rb0 + rg * RB;
    const int kt = jb.kp >> 5;
    const int tb = jb.k0 >> 5, te = jb.k1 >> 5;    // te - tb is even (K slices of 64 k')
    constexpr int TRB = RG * RB;         // row blocks of the tile: the A step stride
    const VT* a = (const VT*)(A + jb.a_off) + (int64_t)(rg * RB) * 128 + lane;
    const VT* b = (const VT*)(B + jb.b_off);
    auto lda = [](const VT* p) -> VT {
        if constexpr (CH == 1) return ld_stream(p);
        else return *p;
    };
    d4_t acc[RB][CTW];
    f4_t ac32[RB][CTW];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < CTW; ++c) {
            acc[r][c] = (d4_t){0, 0, 0, 0};
            ac32[r][c] = (f4_t){0, 0, 0, 0};
        }
    if (te <= tb) {              // empty K slice: its partial output is zero
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int c = 0; c < CTW; ++c) store_c_f32acc(C, jb, rbw + r, c0w + c, lane, acc[r][c]);
        return;
    }
    // this thread's share of B for step t: LDS in lane order, global in column-run order
    auto load_b = [&](VT (&dst)[NU], int t) {
        const int tw = wrap_k(t, kt);
#pragma unroll
        for (int j = 0; j < NU; ++j) {
            const int u = tid + NTH * j, c = u >> 7, rem = u & 127;
            dst[j] = b[((int64_t)c * kt + tw) * 128 + (rem & 64) + bpos(rem & 63)];
        }
    };
    auto store_b = [&](int buf, int sidx, const VT (&src)[NU]) {
#pragma unroll
        for (int j = 0; j < NU; ++j) bs[buf][sidx * STEP_UNITS + tid + NTH * j] = src[j];
    };
    // rings: PFA steps of A and of this thread's share of B in flight
    VT ah[PFA][RB], al[PFA][RB], br[PFA][NU];
#pragma unroll
    for (int u = 0; u < PFA; ++u) {
        const int tl = min(tb + u, te - 1);
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            ah[u][r] = lda(a + (((int64_t)(tl - tb) * TRB + r) * 128));
            al[u][r] = lda(a + (((int64_t)(tl - tb) * TRB + r) * 128 + 64));
        }
        load_b(br[u], tl);
    }
#pragma unroll
    for (int u = 0; u < S; ++u) store_b(0, u, br[u]);
    __syncthreads();
    for (int t0 = tb; t0 < te; t0 += PFA) {
#pragma unroll
        for (int u = 0; u < PFA; ++u) {
            const int t = t0 + u;
            if (t >= te) break;                    // same for every wave of the group
            const int sidx = u % S;                // step inside the group of S
            const int buf = (u / S) & 1;           // groups of S alternate (PFA / S even)
            const VT* bb = bs[buf] + sidx * STEP_UNITS;
            // two column tiles at a time, the three products of a tile interleaved with
            // the other tile's, so dependent MFMAs are 2 RB instructions apart
#pragma unroll
            for (int c = 0; c < CTW; c += 2) {
                const VT bh0 = bb[(c0w + c) * 128 + lane], bl0 = bb[(c0w + c) * 128 + 64 + lane];
                const VT bh1 = bb[(c0w + c + 1) * 128 + lane], bl1 = bb[(c0w + c + 1) * 128 + 64 + lane];
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    ac32[r][c] = mfma_16x16x32(al[u][r], bh0, ac32[r][c]);
                    ac32[r][c + 1] = mfma_16x16x32(al[u][r], bh1, ac32[r][c + 1]);
                }
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    ac32[r][c] = mfma_16x16x32(ah[u][r], bl0, ac32[r][c]);
                    ac32[r][c + 1] = mfma_16x16x32(ah[u][r], bl1, ac32[r][c + 1]);
                }
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    ac32[r][c] = mfma_16x16x32(ah[u][r], bh0, ac32[r][c]);
                    ac32[r][c + 1] = mfma_16x16x32(ah[u][r], bh1, ac32[r][c + 1]);
                }
            }
            // slot u is free (its B went to LDS before this group): refill it PFA ahead
            const int tl = min(t + PFA, te - 1);
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                ah[u][r] = lda(a + (((int64_t)(tl - tb) * TRB + r) * 128));
                al[u][r] = lda(a + (((int64_t)(tl - tb) * TRB + r) * 128 + 64));
            }
            load_b(br[u], tl);
            if (((t - tb + 1) % KCH) == 0 || t + 1 == te) {
#pragma unroll
                for (int r = 0; r < RB; ++r)
#pragma unroll
                    for (int c = 0; c < CTW; ++c) {
#pragma unroll
                        for (int j = 0; j < 4; ++j) acc[r][c][j] += (double)ac32[r][c][j];
                        ac32[r][c] = (f4_t){0, 0, 0, 0};
                    }
            }
            if (sidx == S - 1) {
                if (t + 1 < te) {                  // next group of S steps, from the ring
#pragma unroll
                    for (int v = 1; v <= S; ++v) store_b(buf ^ 1, v - 1, br[(u + v) % PFA]);
                }
                __syncthreads();
            }
        }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < CTW; ++c) store_c_f32acc(C, jb, rbw + r, c0w + c, lane, acc[r][c]);
}

template <typename VT, int RB, int CT, int PFA, int KCH, int S, int NW, int CH = 1>
__global__ void __launch_bounds__(64 * NW) k_gemm_split_lds(const GemmJob* __restrict__ jobs, const unsigned short* __restrict__ A,
        const unsigned short* __restrict__ B, double* __restrict__ C) {
    const GemmJob jb = jobs[blockIdx.x];
    gemm_split_lds_job<VT, RB, CT, PFA, KCH, S, NW, CH>(jb, A, B, C);
}
template <typename VT, int RB, int CT, int PFA, int KCH, int S, int NW, int CH = 1>
__global__ void __launch_bounds__(64 * NW) k_gemm_split_lds_pq(const GemmJob* __restrict__ jobs, int njobs, PqLists q,
        const unsigned short* __restrict__ A, const unsigned short* __restrict__ B, double* __restrict__ C) {
    __shared__ int slot;
    int cur = 0;
    for (int j = pq_next(q, &slot, cur); j < njobs; j = pq_next(q, &slot, cur)) {
        const GemmJob jb = jobs[j];
        gemm_split_lds_job<VT, RB, CT, PFA, KCH, S, NW, CH>(jb, A, B, C);
    }
    pq_done(q);
}

// Row blocks per wave for a given column-tile count (register budget per lane).
static int gemm_rb(int form, int ctmax) {
    // one column tile: 2 row blocks per wave for the FP32 and split products (128-row work
    // groups: finer negligible-block windows and more work groups; measured 3 % faster
    // than 4 on the medium workload), 4 for FP64
    if (form == FBC_FORM_SPLIT_BF16 || form == FBC_FORM_SPLIT_FP16 || form == FBC_FORM_FP32)
        return ctmax <= 1 ? 2 : ctmax <= 2 ? 4 : 2;
    return ctmax <= 2 ? 4 : 2;
}
// Waves per work group (every product kernel as launched runs four).
static int gemm_waves(int, int) { return 4; }
// Rows of a work group's tile (16 per row block): the planner pads rows to whole tiles,
// K' to a multiple of 64, and lays the compact store out in tiles of this height.
int gemm_tile_rows(int form, int ctmax) { return 16 * gemm_rb(form, ctmax) * gemm_waves(form, ctmax); }

template <typename TA>
static void launch_dense(void (*kn)(const GemmJob*, const TA*, const TA*, double*),
                         void (*kp)(const GemmJob*, int, PqLists, const TA*, const TA*, double*),
                         hipStream_t st, const GemmJob* jobs, int njobs, const void* a, const void* b,
                         double* c, const PqLists* q, int threads = 256) {
    if (q)
        hipLaunchKernelGGL(kp, dim3(std::min(njobs, pq_groups_of(kp, threads))), dim3(threads), 0, st, jobs, njobs,
                           *q, (const TA*)a, (const TA*)b, c);
    else
        hipLaunchKernelGGL(kn, dim3(njobs), dim3(threads), 0, st, jobs, (const TA*)a, (const TA*)b, c);
}

// Kernel variants of a product class (form, column tiles) that the autotuner may choose
// from.  They share the tile height (the compact store is laid out in tiles) and the
// arithmetic order, so every variant gives bitwise the same result: variant 0 is the
// default; variant 1 changes the depth of the prefetch ring (FP64, FP32) or the K steps
// per barrier (split products staging B in LDS); variant 2 of those splits the column
// tiles between two halves of eight waves (two waves per SIMD).  The split products with one or two
// column tiles have one variant: their main loop runs whole ring passes, and a 64-k'
// chunk is two of their steps, so the ring cannot be deeper than two steps.
int gemm_variants(int form, int ctmax) {
    if (form == FBC_FORM_SPLIT_FP16 || form == FBC_FORM_SPLIT_BF16) return ctmax <= 2 ? 1 : 3;
    return 2;
}

// Readable shape of a variant: kernel, row blocks per wave, column tiles, ring depth,
// FP32 chunk (K steps), K steps per barrier, waves per group.
std::string gemm_shape(int form, int ctmax, int variant) {
    const int ct = ctmax <= 1 ? 1 : ctmax <= 2 ? 2 : ctmax <= 4 ? 4 : 8;
    const bool alt = variant == 1;
    char buf[96];
    if (form == FBC_FORM_FP64) {
        const int rb = ct <= 2 ? 4 : 2, pf = (ct <= 2) != alt ? 4 : 2;
        snprintf(buf, sizeof buf, "f64 RB=%d CT=%d PF=%d waves=4", rb, ct, pf);
    } else if (form == FBC_FORM_FP32) {
        const int rb = ct == 2 ? 4 : 2, pf = (ct <= 2) != alt ? 4 : 2;
        snprintf(buf, sizeof buf, "f32 RB=%d CT=%d PF=%d KCH=16 waves=4", rb, ct, pf);
    } else if (ct <= 2) {
        const bool f16 = form == FBC_FORM_SPLIT_FP16;
        snprintf(buf, sizeof buf, "split %s RB=%d CT=%d PF=2 KCH=%d waves=4", f16 ? "f16" : "bf16", ct == 2 ? 4 : 2,
                 ct, f16 ? 2 : 8);
    } else {
        const bool f16 = form == FBC_FORM_SPLIT_FP16;
        if (variant == 2)
            snprintf(buf, sizeof buf, "split_lds %s RB=2 CT=%d PFA=4 KCH=%d S=2 waves=8 (column halves)",
                     f16 ? "f16" : "bf16", ct, f16 ? 4 : 8);
        else
            snprintf(buf, sizeof buf, "split_lds %s RB=2 CT=%d PFA=4 KCH=%d S=%d waves=4", f16 ? "f16" : "bf16", ct,
                     f16 ? 4 : 8, alt ? 1 : 2);
    }
    return buf;
}

void launch_gemm(hipStream_t st, int form, const GemmJob* jobs, int njobs, int ctmax,
                 const void* a, const void* b, double* c, const PqLists* q, int variant) {
    if (njobs <= 0) return;
#define GEMM_CASE(KERN, RB, CT, ...)                                                           \
    launch_dense<TA>(KERN<RB, CT, __VA_ARGS__>, KERN##_pq<RB, CT, __VA_ARGS__>, st, jobs, njobs, a, b, c, q)
#define GEMM_PICK(DEF, ALT) do { if (variant == 1) ALT; else DEF; } while (0)
#define GEMM_CASE8(KERN, ...)                                                                  \
    launch_dense<TA>(KERN<__VA_ARGS__, 8, 2>, KERN##_pq<__VA_ARGS__, 8, 2>, st, jobs, njobs, a, b, c, q, 512)
#define GEMM_PICK3(DEF, ALT, CS) do { if (variant == 2) CS; else if (variant == 1) ALT; else DEF; } while (0)
    if (form == FBC_FORM_FP64) {
        typedef double TA;
        if (ctmax <= 1) GEMM_PICK(GEMM_CASE(k_gemm_f64, 4, 1, 4), GEMM_CASE(k_gemm_f64, 4, 1, 2));
        else if (ctmax <= 2) GEMM_PICK(GEMM_CASE(k_gemm_f64, 4, 2, 4), GEMM_CASE(k_gemm_f64, 4, 2, 2));
        else if (ctmax <= 4) GEMM_PICK(GEMM_CASE(k_gemm_f64, 2, 4, 2), GEMM_CASE(k_gemm_f64, 2, 4, 4));
        else GEMM_PICK(GEMM_CASE(k_gemm_f64, 2, 8, 2), GEMM_CASE(k_gemm_f64, 2, 8, 4));
    } else if (form == FBC_FORM_FP32) {
        typedef float TA;
        if (ctmax <= 1) GEMM_PICK(GEMM_CASE(k_gemm_f32, 2, 1, 4, 16), GEMM_CASE(k_gemm_f32, 2, 1, 2, 16));
        else if (ctmax <= 2) GEMM_PICK(GEMM_CASE(k_gemm_f32, 4, 2, 4, 16), GEMM_CASE(k_gemm_f32, 4, 2, 2, 16));
        else if (ctmax <= 4) GEMM_PICK(GEMM_CASE(k_gemm_f32, 2, 4, 2, 16), GEMM_CASE(k_gemm_f32, 2, 4, 4, 16));
        else GEMM_PICK(GEMM_CASE(k_gemm_f32, 2, 8, 2, 16), GEMM_CASE(k_gemm_f32, 2, 8, 4, 16));
    } else if (form == FBC_FORM_SPLIT_FP16) {
        // shorter FP32 chunks: the representation error is ~2^-23, so the FP32 sums must
        // not dominate
        typedef unsigned short TA;
        if (ctmax <= 1) GEMM_CASE(k_gemm_split, h8_t, 2, 1, 2, 2);
        else if (ctmax <= 2) GEMM_CASE(k_gemm_split, h8_t, 4, 2, 2, 2);
        else if (ctmax <= 4)
            GEMM_PICK3(GEMM_CASE(k_gemm_split_lds, h8_t, 2, 4, 4, 4, 2, 4), GEMM_CASE(k_gemm_split_lds, h8_t, 2, 4, 4, 4, 1, 4),
                       GEMM_CASE8(k_gemm_split_lds, h8_t, 2, 4, 4, 4, 2));
        else
            GEMM_PICK3(GEMM_CASE(k_gemm_split_lds, h8_t, 2, 8, 4, 4, 2, 4), GEMM_CASE(k_gemm_split_lds, h8_t, 2, 8, 4, 4, 1, 4),
                       GEMM_CASE8(k_gemm_split_lds, h8_t, 2, 8, 4, 4, 2));
    } else {
        typedef unsigned short TA;
        if (ctmax <= 1) GEMM_CASE(k_gemm_split, bf8_t, 2, 1, 2, 8);
        else if (ctmax <= 2) GEMM_CASE(k_gemm_split, bf8_t, 4, 2, 2, 8);
        else if (ctmax <= 4)
            GEMM_PICK3(GEMM_CASE(k_gemm_split_lds, bf8_t, 2, 4, 4, 8, 2, 4), GEMM_CASE(k_gemm_split_lds, bf8_t, 2, 4, 4, 8, 1, 4),
                       GEMM_CASE8(k_gemm_split_lds, bf8_t, 2, 4, 4, 8, 2));
        else
            GEMM_PICK3(GEMM_CASE(k_gemm_split_lds, bf8_t, 2, 8, 4, 8, 2, 4), GEMM_CASE(k_gemm_split_lds, bf8_t, 2, 8, 4, 8, 1, 4),
                       GEMM_CASE8(k_gemm_split_lds, bf8_t, 2, 8, 4, 8, 2));
    }
#undef GEMM_PICK3
#undef GEMM_CASE8
#undef GEMM_PICK
#undef GEMM_CASE
}

// ------------------------------- offset table (FP64) ------------------------------
// No dense store: the blocks G^(m; n_b - n_i) are gathered from the table of distinct
// column offsets (six symmetric complex components per offset, 96 bytes) into LDS, in
// the FP64 MFMA fragment order, chunk by chunk of 8 interface columns (48 real k').  A
// work group of two waves owns 32 pad columns (96 rows = 6 row blocks, 3 per wave) of
// one mode; the B fragments of the chunk are staged in LDS once for both waves.
#define DT_TB 32
#define DT_TI 8
// Register-prefetch pipeline: the gathers of chunk i+1 are issued right after chunk i has
// been written to LDS, so their latency hides behind the MFMAs of chunk i.  jb.ct_active
// column tiles carry RHS of this cell; the others are skipped.
// F32 (jobs with jb.prec = 1): the same gathered values rounded to FP32 on FP32 MFMA
// 16x16x4 (same operand lanes as the FP64 one), accumulated in FP32 over a chunk of 48
// k' and in FP64 across chunks.
// LDS of the offset-table product, declared once by each kernel and shared by both
// precisions: the A chunk in natural order [row][k'] with an odd row stride (the gathering
// threads' 8-byte writes and the MFMA lanes' 8-byte reads both fall into distinct banks);
// for CT > 2 the chunk's B fragments, staged once for both waves (CT <= 2: each wave keeps
// them in registers, so four work groups fit per CU); the tile's pad columns.
#define DT_AS 49
template <int CT>
struct DtabLds {
    double As[96 * DT_AS];
    double Bs[(CT <= 2 ? 1 : CT * 6 * 128)];   // [ct][p][lane][2]
    int scb[2 * DT_TB];
};
// One job of the offset-table product.  Every thread of the work group calls it with the
// same job (its barriers are uniform); it leaves LDS free for the next job once a barrier
// has followed it.
template <int CT, bool F32>
__device__ inline void dtab_job(DtabLds<CT>& sh, const GemmJob& jb, const double2* __restrict__ tab, int64_t a_base,
                                const double* __restrict__ B, double* __restrict__ C,
                                const CellDev* __restrict__ cells, const int32_t* __restrict__ lut,
                                int d1min, int d2min, int w2, const int32_t* __restrict__ need,
                                int64_t n_off) {
    constexpr int AS = DT_AS;
    double* As = sh.As;
    double* Bs = sh.Bs;
    int* scb = sh.scb;
    if (jb.mb == 0) return;
    const CellDev cd = cells[jb.cell];
    const int nca = jb.ct_active;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int b0 = (jb.rb0 / 6) * DT_TB;
    if (tid < DT_TB) {
        const int b = b0 + tid;
        scb[2 * tid] = b < cd.n_b ? cd.cols_b[2 * b] : 0;
        scb[2 * tid + 1] = b < cd.n_b ? cd.cols_b[2 * b + 1] : 0;
    }
    const double2* tm = tab + (jb.a_off - a_base);
    // generated tables (surrogate form) hold only the first need[t] offsets of table mode t;
    // the rest are zero by definition and are not read
    const int64_t o_lim = need ? (int64_t)need[jb.a_off / (6 * n_off)] : INT64_MAX;
    const double* bm = B + jb.b_off;
    const int kp8 = jb.kp >> 3;
    d4_t acc[3][CT];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[r][c] = (d4_t){0, 0, 0, 0};
    __syncthreads();
    double2 va[2][6];
    double2 vb[CT <= 2 ? 6 : 1][CT <= 2 ? CT : 1];    // next chunk's B fragments (CT <= 2)
    double2 bcur[CT <= 2 ? 6 : 1][CT <= 2 ? CT : 1];  // this chunk's
    const int ni8 = jb.kp / 6;                  // interface columns rounded up to 8
    auto prefetch = [&](int i0u) {
        const int i0 = wrap_k(i0u, ni8);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int q = tid + 128 * h;
            const int bl = q >> 3, il = q & 7;
            const int b = b0 + bl, i = i0 + il;
            if (b < cd.n_b && i < cd.n_i) {
                const int d1 = scb[2 * bl] - cd.cols_i[2 * i] - d1min;
                const int d2 = scb[2 * bl + 1] - cd.cols_i[2 * i + 1] - d2min;
                const int64_t o = lut[(int64_t)d1 * w2 + d2];
                if (o < o_lim) {
                    const double2* src = tm + o * 6;
#pragma unroll
                    for (int s = 0; s < 6; ++s) va[h][s] = src[s];
                } else {
#pragma unroll
                    for (int s = 0; s < 6; ++s) va[h][s] = make_double2(0, 0);
                }
            } else {
#pragma unroll
                for (int s = 0; s < 6; ++s) va[h][s] = make_double2(0, 0);
            }
        }
        if constexpr (CT <= 2) {
            const int p0 = (6 * i0) >> 3;      // physical chunk (i0 wrapped above)
#pragma unroll
            for (int p = 0; p < 6; ++p)
#pragma unroll
                for (int c = 0; c < CT; ++c)
                    vb[p][c] = (c < nca) ? *(const double2*)&bm[((int64_t)c * kp8 + p0 + p) * 128 + 2 * bpos(lane)]
                                         : make_double2(0.0, 0.0);
        }
    };
    prefetch(jb.k0);
    for (int i0 = jb.k0; i0 < jb.k1; i0 += DT_TI) {
        __syncthreads();                          // the previous chunk's MFMAs are done
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int q = tid + 128 * h;
            const int bl = q >> 3, il = q & 7;
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const double2 x = va[h][sym_idx(c, d)];
                    const int row = 3 * bl + c, kq = 6 * il + 2 * d;
                    As[row * AS + kq] = x.x;
                    As[row * AS + kq + 1] = x.y;
                }
        }
        if constexpr (CT <= 2) {
#pragma unroll
            for (int p = 0; p < 6; ++p)
#pragma unroll
                for (int c = 0; c < CT; ++c) bcur[p][c] = vb[p][c];
        } else {
            const int p0 = (6 * wrap_k(i0, ni8)) >> 3;
            for (int e = tid; e < CT * 768; e += 128) {      // LDS in lane order
                const int ct = e / 768, x = e - ct * 768;
                const int pl = x >> 7, l = (x >> 1) & 63, hh = x & 1;
                Bs[e] = (ct < nca) ? bm[((int64_t)ct * kp8 + p0 + pl) * 128 + 2 * bpos(l) + hh] : 0.0;
            }
        }
        if (i0 + DT_TI < jb.k1) prefetch(i0 + DT_TI);
        __syncthreads();
        f4_t a32[3][CT];
        if constexpr (F32) {
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < CT; ++c) a32[r][c] = (f4_t){0, 0, 0, 0};
        }
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            double2 av[3], bv[CT];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                // lane l holds A[16 rb + l%16][8 p + 4 h + l/16], h = 0, 1 (FP64 16x16x4 order)
                const double* ap = &As[(16 * (3 * wave + r) + (lane & 15)) * AS + 8 * p + (lane >> 4)];
                av[r] = make_double2(ap[0], ap[4]);
            }
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                if constexpr (CT <= 2) bv[c] = bcur[p][c];
                else bv[c] = *(const double2*)&Bs[(c * 6 + p) * 128 + 2 * lane];
            }
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int r = 0; r < 3; ++r)
#pragma unroll
                    for (int c = 0; c < CT; ++c)
                        if (c < nca) {
                            if constexpr (F32)
                                a32[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                    (float)(h ? av[r].y : av[r].x), (float)(h ? bv[c].y : bv[c].x), a32[r][c], 0, 0,
                                    0);
                            else
                                acc[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(h ? av[r].y : av[r].x,
                                                                                 h ? bv[c].y : bv[c].x,
                                                                                 acc[r][c], 0, 0, 0);
                        }
        }
        if constexpr (F32) {
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < CT; ++c)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[r][c][j] += (double)a32[r][c][j];
        }
    }
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < CT; ++c)
            if (c < nca) {
                if constexpr (F32) store_c_f32acc(C, jb, jb.rb0 + 3 * wave + r, c, lane, acc[r][c]);
                else store_c_f64(C, jb, jb.rb0 + 3 * wave + r, c, lane, acc[r][c]);
            }
}

// MIX = 0: every job on FP64 MFMA; MIX = 1 (options.table_fp32): each job in its own
// precision (jb.prec).  Separate instantiations, so that the FP64 kernel keeps its own
// register allocation.
template <int CT, int MIX>
__device__ inline void dtab_any(DtabLds<CT>& sh, const GemmJob& jb, const double2* __restrict__ tab, int64_t a_base,
                                const double* __restrict__ B, double* __restrict__ C,
                                const CellDev* __restrict__ cells, const int32_t* __restrict__ lut, int d1min,
                                int d2min, int w2, const int32_t* __restrict__ need, int64_t n_off) {
    if (MIX && jb.prec) dtab_job<CT, true>(sh, jb, tab, a_base, B, C, cells, lut, d1min, d2min, w2, need, n_off);
    else dtab_job<CT, false>(sh, jb, tab, a_base, B, C, cells, lut, d1min, d2min, w2, need, n_off);
}

// One work group per job, in list order.
template <int CT, int MIX>
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(CT == 2 ? 2 : 1)))
k_gemm_dtab(const GemmJob* __restrict__ jobs, const double2* __restrict__ tab, int64_t a_base,
            const double* __restrict__ B, double* __restrict__ C, const CellDev* __restrict__ cells,
            const int32_t* __restrict__ lut, int d1min, int d2min, int w2,
            const int32_t* __restrict__ need, int64_t n_off) {
    __shared__ DtabLds<CT> sh;
    const GemmJob jb = jobs[blockIdx.x];
    dtab_any<CT, MIX>(sh, jb, tab, a_base, B, C, cells, lut, d1min, d2min, w2, need, n_off);
}

// Persistent form (work queue as for the dense products).
template <int CT, int MIX>
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(CT == 2 ? 2 : 1)))
k_gemm_dtab_pq(const GemmJob* __restrict__ jobs, int njobs, PqLists q,
               const double2* __restrict__ tab, int64_t a_base, const double* __restrict__ B,
               double* __restrict__ C, const CellDev* __restrict__ cells,
               const int32_t* __restrict__ lut, int d1min, int d2min, int w2,
               const int32_t* __restrict__ need, int64_t n_off) {
    __shared__ int slot;
    __shared__ DtabLds<CT> sh;
    int cur = 0;
    for (int j = pq_next(q, &slot, cur); j < njobs; j = pq_next(q, &slot, cur)) {
        const GemmJob jb = jobs[j];
        dtab_any<CT, MIX>(sh, jb, tab, a_base, B, C, cells, lut, d1min, d2min, w2, need, n_off);
    }
    pq_done(q);
}

void launch_gemm_dtab(hipStream_t st, const GemmJob* jobs, int njobs, int ct, const double2* tab,
                      int64_t a_base, const double* b, double* c, const CellDev* cells,
                      const int32_t* lut, int d1min, int d2min, int w2, const int32_t* need,
                      int64_t n_off, const PqLists* q, int mixed) {
    if (njobs <= 0) return;
    dim3 blk(128);
    if (q) {
#define PQ_CASE(CT, MIX)                                                                             \
    hipLaunchKernelGGL((k_gemm_dtab_pq<CT, MIX>), dim3(std::min(njobs, pq_groups_of(k_gemm_dtab_pq<CT, MIX>, 128))), blk, 0, \
                       st, jobs, njobs, *q, tab, a_base, b, c, cells, lut, d1min, d2min, w2, need, n_off)
#define PQ_CT(CT) do { if (mixed) PQ_CASE(CT, 1); else PQ_CASE(CT, 0); } while (0)
        switch (ct) {
            case 1: PQ_CT(1); break;
            case 2: PQ_CT(2); break;
            case 4: PQ_CT(4); break;
            default: PQ_CT(8); break;
        }
#undef PQ_CT
#undef PQ_CASE
        return;
    }
    dim3 grid(njobs);
#define DT_CASE(CT, MIX)                                                                              \
    hipLaunchKernelGGL((k_gemm_dtab<CT, MIX>), grid, blk, 0, st, jobs, tab, a_base, b, c, cells, lut, d1min, d2min, \
                       w2, need, n_off)
#define DT_CT(CT) do { if (mixed) DT_CASE(CT, 1); else DT_CASE(CT, 0); } while (0)
    switch (ct) {
        case 1: DT_CT(1); break;
        case 2: DT_CT(2); break;
        case 4: DT_CT(4); break;
        default: DT_CT(8); break;
    }
#undef DT_CT
#undef DT_CASE
}
