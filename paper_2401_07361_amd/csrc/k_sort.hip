// Stable LSD radix sort of 64-bit keys over a bit range, 8 bits per pass.
// Used to order particles by leaf key (ties by input index, which is packed
// in the low bits) and interaction lists by (target, type, source).
//
// Per pass: (1) per-tile digit histograms, (2) one exclusive scan over
// (digit, tile), (3) a stable scatter: inside a tile, keys are ranked in
// index order with wave ballots (lanes holding the same digit) and per-wave
// digit counts in LDS.  The key count may live in device memory (n_bound is
// then only the capacity that sizes the grid), so no host synchronisation is
// needed between the traversal and the sort.
#include "common.hpp"

namespace stc {

namespace {

constexpr int RS_THREADS = 256;
constexpr int RS_IPT = 16;
constexpr int RS_TILE = RS_THREADS * RS_IPT;

__device__ __forceinline__ u32 load_n(const u32* d_n, u32 n_bound) {
    if (d_n == nullptr) return n_bound;
    u32 n = *d_n;
    return n < n_bound ? n : n_bound;
}

__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const u64* __restrict__ keys, const u32* d_n,
                                                         u32 n_bound, int shift, u32* __restrict__ hist,
                                                         int nblocks) {
    __shared__ u32 h[256];
    const int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const u32 n = load_n(d_n, n_bound);
    const u64 base = (u64)blockIdx.x * RS_TILE;
    if (base < n) {
        for (int r = 0; r < RS_IPT; ++r) {
            const u64 i = base + (u64)r * RS_THREADS + tid;
            if (i < n) atomicAdd(&h[(u32)(keys[i] >> shift) & 255u], 1u);
        }
    }
    __syncthreads();
    hist[(size_t)tid * nblocks + blockIdx.x] = h[tid];
}

// Exclusive scan over (digit, tile) in digit-major order, for the tiles in use.
__global__ __launch_bounds__(1024) void k_rs_scan(u32* __restrict__ hist, const u32* d_n, u32 n_bound,
                                                  int nblocks) {
    __shared__ u32 part[1024];
    const int tid = threadIdx.x;
    const u32 n = load_n(d_n, n_bound);
    const u32 used = (n + RS_TILE - 1) / RS_TILE;
    const u64 total = (u64)256 * used;
    const u64 per = (total + 1023) / 1024;
    const u64 lo = (u64)tid * per;
    const u64 hi = lo + per < total ? lo + per : total;
    u32 s = 0;
    for (u64 e = lo; e < hi; ++e) {
        const u64 d = e / used, b = e % used;
        s += hist[d * nblocks + b];
    }
    part[tid] = s;
    __syncthreads();
    // inclusive scan of the 1024 partial sums (Hillis-Steele)
    for (int off = 1; off < 1024; off <<= 1) {
        u32 v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    u32 run = tid > 0 ? part[tid - 1] : 0;
    for (u64 e = lo; e < hi; ++e) {
        const u64 d = e / used, b = e % used;
        const u32 v = hist[d * nblocks + b];
        hist[d * nblocks + b] = run;
        run += v;
    }
}

__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(const u64* __restrict__ in, u64* __restrict__ out,
                                                            const u32* d_n, u32 n_bound, int shift,
                                                            const u32* __restrict__ hist, int nblocks) {
    __shared__ u32 digit_base[256];
    __shared__ u32 wcnt[4][256];
    __shared__ u32 run[256];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const u32 n = load_n(d_n, n_bound);
    const u64 base = (u64)blockIdx.x * RS_TILE;
    if (base >= n) return;  // uniform over the block
    digit_base[tid] = hist[(size_t)tid * nblocks + blockIdx.x];
    run[tid] = 0;
    const u64 lt = lanemask_lt();
    for (int r = 0; r < RS_IPT; ++r) {
        const u64 i = base + (u64)r * RS_THREADS + tid;
        const bool valid = i < n;
        const u64 key = valid ? in[i] : 0;
        const u32 d = (u32)(key >> shift) & 255u;
        for (int k = 0; k < 4; ++k) wcnt[k][tid] = 0;
        __syncthreads();
        u64 m = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const u64 bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const u32 rank = (u32)__popcll(m & lt);
        if (valid && rank == 0) wcnt[w][d] = (u32)__popcll(m);
        __syncthreads();
        {
            const u32 c0 = wcnt[0][tid], c1 = wcnt[1][tid], c2 = wcnt[2][tid], c3 = wcnt[3][tid];
            const u32 r0 = run[tid];
            wcnt[0][tid] = r0;
            wcnt[1][tid] = r0 + c0;
            wcnt[2][tid] = r0 + c0 + c1;
            wcnt[3][tid] = r0 + c0 + c1 + c2;
            run[tid] = r0 + c0 + c1 + c2 + c3;
        }
        __syncthreads();
        if (valid) out[(u64)digit_base[d] + wcnt[w][d] + rank] = key;
        __syncthreads();
    }
}

}  // namespace

void radix_sort(hipStream_t s, u64* keys, u64* tmp, const u32* d_n, u32 n_bound, int bit_lo, int bit_hi,
                SortScratch scratch, u64** result) {
    u64* a = keys;
    u64* b = tmp;
    const int nblocks = (int)((n_bound + RS_TILE - 1) / RS_TILE);
    if (n_bound == 0 || nblocks > scratch.max_blocks) {
        *result = keys;
        return;
    }
    for (int sh = bit_lo; sh < bit_hi; sh += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3(nblocks), dim3(RS_THREADS), 0, s, a, d_n, n_bound, sh,
                           scratch.hist, nblocks);
        hipLaunchKernelGGL(k_rs_scan, dim3(1), dim3(1024), 0, s, scratch.hist, d_n, n_bound, nblocks);
        hipLaunchKernelGGL(k_rs_scatter, dim3(nblocks), dim3(RS_THREADS), 0, s, a, b, d_n, n_bound, sh,
                           scratch.hist, nblocks);
        u64* t = a;
        a = b;
        b = t;
    }
    *result = a;
}

}  // namespace stc
