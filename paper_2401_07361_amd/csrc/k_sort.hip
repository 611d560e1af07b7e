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

__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(SortBatch sb, u32 n_bound, int shift, u32* __restrict__ hist_all,
                                                         int nblocks) {
    __shared__ u32 h[256];
    const int tid = threadIdx.x;
    const int y = blockIdx.y;
    const u64* __restrict__ keys = sb.in[y];
    const u32* d_n = sb.dn[y];
    u32* __restrict__ hist = hist_all + (size_t)y * 256 * nblocks;
    const u32 n = load_n(d_n, n_bound);
    const u64 base = (u64)blockIdx.x * RS_TILE;
    if (base >= n) return;  // tiles past the key count are never scanned
    h[tid] = 0;
    u32 dg[RS_IPT];
#pragma unroll
    for (int r = 0; r < RS_IPT; ++r) {
        const u64 i = base + (u64)r * RS_THREADS + tid;
        dg[r] = i < n ? ((u32)(keys[i] >> shift) & 255u) : 256u;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RS_IPT; ++r)
        if (dg[r] < 256u) atomicAdd(&h[dg[r]], 1u);
    __syncthreads();
    hist[(size_t)tid * nblocks + blockIdx.x] = h[tid];
}

// Per-digit exclusive scan over the tiles in use: workgroup d scans
// hist[d][0..used) in coalesced chunks of 256 and stores the digit total.
// The scatter adds the exclusive prefix over digit totals.
__global__ __launch_bounds__(256) void k_rs_scan(SortBatch sb, u32* __restrict__ hist_all, u32* __restrict__ totals_all,
                                                 u32 n_bound, int nblocks) {
    __shared__ u32 part[256];
    const int tid = threadIdx.x;
    const int d = blockIdx.x;
    const int y = blockIdx.y;
    const u32* d_n = sb.dn[y];
    u32* __restrict__ hist = hist_all + (size_t)y * 256 * nblocks;
    u32* __restrict__ totals = totals_all + 256 * y;
    const u32 n = load_n(d_n, n_bound);
    const u32 used = (n + RS_TILE - 1) / RS_TILE;
    u32* h = hist + (size_t)d * nblocks;
    u32 carry = 0;
    for (u32 b0 = 0; b0 < used; b0 += 256) {
        const u32 b = b0 + tid;
        const u32 v = b < used ? h[b] : 0u;
        part[tid] = v;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const u32 t = tid >= off ? part[tid - off] : 0u;
            __syncthreads();
            part[tid] += t;
            __syncthreads();
        }
        if (b < used) h[b] = carry + part[tid] - v;
        carry += part[255];
        __syncthreads();
    }
    if (tid == 0) totals[d] = carry;
}

__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(SortBatch sb, u32 n_bound, int shift,
                                                            const u32* __restrict__ hist_all,
                                                            const u32* __restrict__ totals_all, int nblocks) {
    const int y = blockIdx.y;
    const u64* __restrict__ in = sb.in[y];
    u64* __restrict__ out = sb.out[y];
    const u32* d_n = sb.dn[y];
    const u32* __restrict__ hist = hist_all + (size_t)y * 256 * nblocks;
    const u32* __restrict__ totals = totals_all + 256 * y;
    __shared__ u32 digit_base[256];
    __shared__ u32 wcnt[4][256];
    __shared__ u32 run[256];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const u32 n = load_n(d_n, n_bound);
    const u64 base = (u64)blockIdx.x * RS_TILE;
    if (base >= n) return;  // uniform over the block
    // exclusive prefix of the digit totals (Hillis-Steele in LDS)
    const u32 tot = totals[tid];
    run[tid] = tot;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const u32 t = tid >= off ? run[tid - off] : 0u;
        __syncthreads();
        run[tid] += t;
        __syncthreads();
    }
    digit_base[tid] = run[tid] - tot + hist[(size_t)tid * nblocks + blockIdx.x];
    __syncthreads();
    run[tid] = 0;
    const u64 lt = lanemask_lt();
    u64 keys[RS_IPT];  // all loads of the tile in flight at once
#pragma unroll
    for (int r = 0; r < RS_IPT; ++r) {
        const u64 i = base + (u64)r * RS_THREADS + tid;
        keys[r] = i < n ? in[i] : 0;
    }
#pragma unroll
    for (int r = 0; r < RS_IPT; ++r) {
        const u64 i = base + (u64)r * RS_THREADS + tid;
        const bool valid = i < n;
        const u64 key = keys[r];
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

void radix_sort_batch(hipStream_t s, int nb, u64* const* keys, u64* const* tmp, const u32* const* d_n, u32 n_bound,
                      int bit_lo, int bit_hi, SortScratch scratch, u64** result) {
    const int nblocks = (int)((n_bound + RS_TILE - 1) / RS_TILE);
    SortBatch sb{};
    u64* a[2] = {keys[0], nb > 1 ? keys[1] : nullptr};
    u64* b[2] = {tmp[0], nb > 1 ? tmp[1] : nullptr};
    for (int y = 0; y < nb; ++y) sb.dn[y] = d_n[y];
    if (n_bound == 0 || nblocks > scratch.max_blocks || nb < 1 || nb > 2) {
        for (int y = 0; y < nb; ++y) result[y] = keys[y];
        return;
    }
    for (int sh = bit_lo; sh < bit_hi; sh += 8) {
        for (int y = 0; y < nb; ++y) {
            sb.in[y] = a[y];
            sb.out[y] = b[y];
        }
        hipLaunchKernelGGL(k_rs_hist, dim3(nblocks, nb), dim3(RS_THREADS), 0, s, sb, n_bound, sh, scratch.hist, nblocks);
        hipLaunchKernelGGL(k_rs_scan, dim3(256, nb), dim3(256), 0, s, sb, scratch.hist, scratch.totals, n_bound,
                           nblocks);
        hipLaunchKernelGGL(k_rs_scatter, dim3(nblocks, nb), dim3(RS_THREADS), 0, s, sb, n_bound, sh, scratch.hist,
                           scratch.totals, nblocks);
        for (int y = 0; y < nb; ++y) {
            u64* t = a[y];
            a[y] = b[y];
            b[y] = t;
        }
    }
    for (int y = 0; y < nb; ++y) result[y] = a[y];
}

void radix_sort(hipStream_t s, u64* keys, u64* tmp, const u32* d_n, u32 n_bound, int bit_lo, int bit_hi,
                SortScratch scratch, u64** result) {
    u64* k[1] = {keys};
    u64* t[1] = {tmp};
    const u32* n[1] = {d_n};
    radix_sort_batch(s, 1, k, t, n, n_bound, bit_lo, bit_hi, scratch, result);
}

}  // namespace stc
