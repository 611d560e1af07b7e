// Stable LSD radix sort of 64-bit keys over a bit range, 8 bits per pass.
// Used to order particles by leaf key (ties by input index, which is packed
// in the low bits) and interaction lists by (target, type, source).
//
// One-sweep form: k_os_hist counts the first pass's digits; then one kernel
// per pass, which also counts its tile's digits of the next pass (the keys
// are in registers anyway).  A pass kernel takes its tile number
// from an atomic counter (tiles are numbered in the order they start), ranks
// the tile's 4096 keys stably (each of its sixteen waves ranks its contiguous
// 256 keys with ballots and wave-private running counts in LDS, then one
// prefix over the waves), publishes its digit counts, and looks back over the
// earlier tiles' published counts to find where its keys go (decoupled
// look-back: a tile adds the counts of predecessors that only published their
// own counts and stops at the first that published its inclusive prefix).  A
// tile waits only on tiles that started before it, so every wait ends; the
// spin is also bounded, and a tile that exceeds the bound sets an error flag
// and goes on.
//
// The pass grid is persistent (at most the workgroups resident at once, each
// taking tiles until none is left), so that a capacity-sized array of which
// only a part is used costs no launches of idle workgroups.
//
// A pass is latency-bound (18-20 us for up to a few million keys): the ballot
// rounds of the ranking form a dependent chain per wave, so a tile is spread
// over sixteen waves of four keys (four waves per SIMD, four rounds each);
// larger tiles lengthen the ranking, smaller ones the look-back chain and the
// serialised tile-counter atomics.
//
// Status words: epoch (30 bits) | state (2 bits: 1 own count, 2 inclusive
// prefix) | count (32 bits).  The epoch of a pass comes from a device counter
// that k_os_hist advances, so statuses left by an earlier sort (or an earlier
// replay of a captured graph) never match.  The digit histograms and tile
// counters must be zero when a sort starts (the callers clear them together
// with their other per-evaluation counters); each histogram is kept in
// kSortCopies copies (workgroup b adds to copy b % kSortCopies) so that the
// atomics of many workgroups do not all meet on 256 addresses.  The key count may live in
// device memory (n_bound then only sizes the grid), so no host
// synchronisation is needed between the traversal and the sort.
#include <algorithm>

#include "common.hpp"

namespace stc {

namespace {

constexpr int OS_THREADS = 256;                 // first-pass histogram; a thread per digit in a pass
constexpr int OS_WAVES = 16;                    // waves of a pass workgroup
constexpr int OS_PASS_THREADS = 64 * OS_WAVES;  // 1024
constexpr int OS_IPT = 4;                       // keys per thread
constexpr int OS_TILE = OS_PASS_THREADS * OS_IPT;  // 4096
constexpr int OS_WAVE_KEYS = 64 * OS_IPT;     // a wave's contiguous sixteenth of the tile
// a look-back poll takes about a microsecond: this bound (a few ms per tile)
// is far above any real wait and keeps even a broken chain of tiles short
constexpr u32 OS_SPIN_LIMIT = 1u << 12;
constexpr u64 OS_AGG = 1ull << 32, OS_INC = 2ull << 32;
constexpr int OS_WIN = 8;  // look-back window

__device__ __forceinline__ u32 load_n(const u32* d_n, u32 n_bound) {
    if (d_n == nullptr) return n_bound;
    u32 n = *d_n;
    return n < n_bound ? n : n_bound;
}

__device__ __forceinline__ u32 pass_epoch(u32 base, int p) { return ((base + (u32)p) % 0x3fffffffu) + 1u; }

// Digit histogram of the first pass, ghist[y][0][d] (each pass kernel
// counts the next pass's digits of its tile); block 0 advances the epoch
// counter by the number of passes.
__global__ __launch_bounds__(OS_THREADS) void k_os_hist(SortBatch sb, u32 n_bound, int bit_lo, int passes,
                                                         u32* __restrict__ zero_region, u32* __restrict__ epoch) {
    __shared__ u32 h[256];
    const int tid = threadIdx.x, y = blockIdx.y;
    const u64* __restrict__ keys = sb.in[y];
    const u32 n = load_n(sb.dn[y], n_bound);
    u32* __restrict__ ghist = zero_region + (size_t)y * kSortMaxPasses * kSortCopies * 256 +
                              (blockIdx.x % kSortCopies) * 256;
    if (blockIdx.x == 0 && tid == 0) epoch[y] += (u32)passes;
    h[tid] = 0u;
    __syncthreads();
    const u64 stride = (u64)gridDim.x * OS_THREADS;
    for (u64 i = (u64)blockIdx.x * OS_THREADS + tid; i < n; i += stride)
        atomicAdd(&h[(u32)(keys[i] >> bit_lo) & 255u], 1u);
    __syncthreads();
    if (h[tid]) atomicAdd(&ghist[tid], h[tid]);
}

__global__ __launch_bounds__(OS_PASS_THREADS) void k_os_pass(SortBatch sb, u32 n_bound, int shift, int p, int passes,
                                                         u32* __restrict__ zero_region,
                                                         u64* __restrict__ status_all, int max_tiles,
                                                         const u32* __restrict__ epoch, u32* __restrict__ err) {
    __shared__ u32 wrun[OS_WAVES][256];  // per wave: running digit counts, then their prefix over waves
    __shared__ u32 dpre[256];     // global exclusive prefix over digits, then the tile's base per digit
    __shared__ u32 hnext[256];    // the tile's digits of the next pass
    __shared__ u32 tile_sh;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, y = blockIdx.y;
    const u64* __restrict__ in = sb.in[y];
    u64* __restrict__ out = sb.out[y];
    const u32 n = load_n(sb.dn[y], n_bound);
    const u32 used = (n + OS_TILE - 1) / OS_TILE;
    u32* __restrict__ ghist = zero_region + ((size_t)y * kSortMaxPasses + p) * kSortCopies * 256;
    u32* __restrict__ gnext = ghist + kSortCopies * 256 + (blockIdx.x % kSortCopies) * 256;  // next pass, one copy
    u32* __restrict__ tctr = zero_region + kSortHistWords + y * kSortMaxPasses + p;
    u64* __restrict__ status = status_all + (size_t)y * max_tiles * 256;
    const u32 ep = pass_epoch(epoch[y] - (u32)passes, p);  // k_os_hist advanced the counter by `passes`
    // a persistent grid of at most the resident workgroups: each takes tile
    // numbers from the counter, in the order in which it is ready for them,
    // until they run out (a tile's look-back waits only on lower numbers,
    // each held by a workgroup that completes it without waiting on higher
    // ones)
    const bool dig = tid < 256;  // the first four waves also work per digit (thread = digit)
    u32 v = 0;  // digit tid's global count: loads issued before the tile-counter atomic (latencies overlap)
    if (dig) {
#pragma unroll
        for (int c = 0; c < kSortCopies; ++c) v += ghist[c * 256 + tid];
    }
    u32 my_tile = 0;
    if (tid == 0) my_tile = atomicAdd(tctr, 1u);
    // exclusive prefix of the global digit counts (the same for every tile)
    u32 gpre;
    {
        u32 incl = v;
        for (int o = 1; o < 64; o <<= 1) {
            const u32 t = __shfl_up(incl, o, 64);
            if (lane >= o) incl += t;
        }
        if (dig && lane == 63) dpre[w] = incl;  // wave totals
        __syncthreads();
        u32 base = 0;
        for (int k = 0; k < w && dig; ++k) base += dpre[k];
        gpre = base + incl - v;
    }
    for (;;) {
        wrun[w][lane] = 0u;
        wrun[w][lane + 64] = 0u;
        wrun[w][lane + 128] = 0u;
        wrun[w][lane + 192] = 0u;
        if (dig) hnext[tid] = 0u;
        if (tid == 0) tile_sh = my_tile;
        __syncthreads();
        const u32 tile = tile_sh;
        if (tile >= used) break;  // uniform
        // keys of this wave's sixteenth of the tile, all loads in flight at once
        const u64 q0 = (u64)tile * OS_TILE + (u64)w * OS_WAVE_KEYS;
        u64 keys[OS_IPT];
#pragma unroll
        for (int r = 0; r < OS_IPT; ++r) {
            const u64 i = q0 + (u64)r * 64 + lane;
            keys[r] = i < n ? in[i] : 0ull;
        }
        // stable ranks inside the wave (rounds in key order)
        const u64 lt = lanemask_lt();
        u32 rank[OS_IPT];
    #pragma unroll
        for (int r = 0; r < OS_IPT; ++r) {
            const bool valid = q0 + (u64)r * 64 + lane < n;
            const u32 d = (u32)(keys[r] >> shift) & 255u;
            u64 m = __ballot(valid);
    #pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1u;
                const u64 bb = __ballot(bit);
                m &= bit ? bb : ~bb;
            }
            if (p + 1 < passes) {
                const u32 d2 = (u32)(keys[r] >> (shift + 8)) & 255u;
                const u32 d20 = (u32)__shfl(d2, 0, 64);
                const u64 act = __ballot(valid);
                if (__ballot(valid && d2 == d20) == act) {
                    if (lane == 0 && act) atomicAdd(&hnext[d20], (u32)__popcll(act));
                } else if (valid) {
                    atomicAdd(&hnext[d2], 1u);
                }
            }
            const u32 before = valid ? wrun[w][d] : 0u;
            const u32 rr = (u32)__popcll(m & lt);
            // every lane has read its digit's count before any leader writes it
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (valid && rr == 0) wrun[w][d] = before + (u32)__popcll(m);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            rank[r] = before + rr;
        }
        __syncthreads();
        if (dig && p + 1 < passes && hnext[tid]) atomicAdd(&gnext[tid], hnext[tid]);
        // per digit (thread = digit): prefix over the waves, the tile's count
        u32 cnt = 0;
        if (dig) {
#pragma unroll
            for (int k = 0; k < OS_WAVES; ++k) {
                const u32 t = wrun[k][tid];
                wrun[k][tid] = cnt;
                cnt += t;
            }
        }
        // publish, look back, publish the inclusive prefix
        u64* my = status + (size_t)tile * 256 + tid;
        const u64 tag = (u64)ep << 34;
        u32 excl = 0;
        if (!dig) {
        } else if (tile == 0) {
            __hip_atomic_store(my, tag | OS_INC | cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(my, tag | OS_AGG | cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // predecessors read OS_WIN at a time (one memory round trip per
            // window), taken in order: add own counts, stop at an inclusive
            // prefix, re-read from the first tile that has not published yet
            int j = (int)tile - 1;
            u32 spins = 0;
            bool done = false;
            while (!done && j >= 0) {
                u64 st[OS_WIN];
    #pragma unroll
                for (int t = 0; t < OS_WIN; ++t)
                    st[t] = (j - t >= 0) ? __hip_atomic_load(status + (size_t)(j - t) * 256 + tid, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT)
                                         : 0ull;
                int adv = 0;
                bool stall = false;
    #pragma unroll
                for (int t = 0; t < OS_WIN; ++t) {
                    if (done || stall || j - t < 0) continue;
                    const u32 sep = (u32)(st[t] >> 34), state = (u32)(st[t] >> 32) & 3u;
                    if (sep != ep || state == 0u) {
                        stall = true;
                        continue;
                    }
                    excl += (u32)st[t];
                    ++adv;
                    if (state == 2u) done = true;
                }
                j -= adv;
                if (stall && !done) {
                    if (++spins > OS_SPIN_LIMIT) {
                        atomicOr(err, 1u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            __hip_atomic_store(my, tag | OS_INC | (excl + cnt), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (dig) dpre[tid] = gpre + excl;
        if (tid == 0) my_tile = atomicAdd(tctr, 1u);  // the next tile (this one has published its prefix)
        __syncthreads();
#pragma unroll
        for (int r = 0; r < OS_IPT; ++r) {
            if (q0 + (u64)r * 64 + lane < n) {
                const u32 d = (u32)(keys[r] >> shift) & 255u;
                const u64 pos = (u64)dpre[d] + wrun[w][d] + rank[r];
                if (pos < n_bound) out[pos] = keys[r];  // always true unless a look-back gave up
            }
        }
        __syncthreads();  // the LDS counts are read before the next tile clears them
    }
}

// workgroups of k_os_pass resident on the current device at once (cached
// per device; at least one)
int os_pass_resident() {
    static int cached[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        (void)hipGetLastError();
        dev = -1;
    }
    if (dev >= 0 && cached[dev] > 0) return cached[dev];
    int bpc = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, k_os_pass, OS_PASS_THREADS, 0) != hipSuccess || bpc < 1) {
        (void)hipGetLastError();
        bpc = 1;
    }
    if (dev < 0 || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) {
        (void)hipGetLastError();
        cus = 1;
    }
    const int r = bpc * cus;
    if (dev >= 0) cached[dev] = r;
    return r;
}

}  // namespace

int sort_passes(int bit_lo, int bit_hi) { return bit_hi > bit_lo ? (bit_hi - bit_lo + 7) / 8 : 0; }

void radix_sort_batch(hipStream_t s, int nb, u64* const* keys, u64* const* tmp, const u32* const* d_n, u32 n_bound,
                      int bit_lo, int bit_hi, SortScratch scratch, u64** result) {
    const int tiles = (int)((n_bound + OS_TILE - 1) / OS_TILE);
    const int passes = sort_passes(bit_lo, bit_hi);
    for (int y = 0; y < nb; ++y) result[y] = keys[y];
    if (n_bound == 0 || passes == 0 || passes > kSortMaxPasses || tiles > scratch.max_tiles || nb < 1 || nb > 2)
        return;
    SortBatch sb{};
    u64* a[2] = {keys[0], nb > 1 ? keys[1] : nullptr};
    u64* b[2] = {tmp[0], nb > 1 ? tmp[1] : nullptr};
    for (int y = 0; y < nb; ++y) {
        sb.dn[y] = d_n[y];
        sb.in[y] = a[y];
    }
    const unsigned hb = (unsigned)(tiles < 256 ? tiles : 256);
    hipLaunchKernelGGL(k_os_hist, dim3(hb, nb), dim3(OS_THREADS), 0, s, sb, n_bound, bit_lo, passes, scratch.zero,
                       scratch.epoch);
    // persistent grid: the resident workgroups shared among the nb arrays
    const int per = std::max(1, os_pass_resident() / nb);
    const unsigned grid = (unsigned)std::min(tiles, per);
    for (int p = 0; p < passes; ++p) {
        for (int y = 0; y < nb; ++y) {
            sb.in[y] = a[y];
            sb.out[y] = b[y];
        }
        hipLaunchKernelGGL(k_os_pass, dim3(grid, nb), dim3(OS_PASS_THREADS), 0, s, sb, n_bound, bit_lo + 8 * p, p,
                           passes, scratch.zero, scratch.status, scratch.max_tiles, scratch.epoch, scratch.err);
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
