// Shared device helpers and internal declarations of the HIP library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "geometry.hpp"

namespace stc {

using u8 = uint8_t;
using u16 = uint16_t;
using u32 = uint32_t;
using u64 = uint64_t;
using i32 = int32_t;
using i64 = int64_t;

constexpr double kInv4Pi = 0.07957747154594767;  // 1 / (4 pi)
constexpr int kMaxDegree = 14;
constexpr int kMaxNp = (kMaxDegree + 1) * (kMaxDegree + 2) / 2;  // 120
constexpr int UP_CHUNK = 2048;  // particles per upward-pass item
constexpr int UP_BATCH = 8;     // big nodes per workgroup when the upward pass finishes
constexpr int kMaxLevels = 12;  // deepest tree level

// Ensembles (batched evaluation): up to kMaxMembers independent particle
// sets share one launch per phase.  Node ids carry the member above the local
// id, id = (member << NB) | local, with local = 20 (4^l - 1)/3 + key as for a
// single tree and NB = bits of the local node count; particle leaf keys carry
// it the same way above their 2 L + 5 bits.  Geometry is indexed by local id.
constexpr int kMaxMembers = 64;

// member m owns particles [off[m], off[m+1]) of the concatenated arrays
struct MemberOffsets {
    i64 off[kMaxMembers + 1];
    int m;
};

// flag slots in the context's u32 flag array
enum Flag : int {
    F_NONFINITE = 0,  // a particle position lies in no root face
    F_SLOTS = 1,      // more nodes with proxy charges than storage slots
    F_SLOT_CTR = 2,   // next free storage slot (counter)
    F_BIN_EXACT = 3,  // points queued for exact point location
    F_ITEMS = 4,      // upward-pass items (pieces of big nodes' particle ranges)
    F_SORT_SPIN = 5,  // a sort's look-back exceeded its spin bound
    F_NONFINITE_CHARGE = 6,  // a charge zeta A is NaN or infinite
    F_LEVEL = 8,      // F_LEVEL + l: nodes of level l with more than N_T particles (list length)
    F_COUNT = 24
};

// counter slots in the context's u32 counter array
enum Counter : int {
    C_TLIST = 0,      // entries in the target-particle list (PP + PC)
    C_NLIST = 1,      // entries in the target-proxy list (CP + CC)
    C_PP = 2, C_PC = 3, C_CP = 4, C_CC = 5,
    C_OVERFLOW = 6,   // set to 1 when any list or frontier outgrows capacity
    C_CAND = 7,       // candidate pairs of a gated traversal
    C_FRONT = 16,     // C_FRONT + k: frontier length at traversal iteration k
    C_FRONT2 = 64,    // the same for the fallback traversal of rejected candidates
    C_COUNT = 128
};

// An interpolation point of a node with its proxy charge (written by the
// upward pass for every node with more than N_T particles).
struct Prox {
    double x, y, z, w;
};

// Interpolation tables on the device.
struct RefDev {
    const double* points;  // np x 3
    const double* vinv;    // np x np, [k*np + m]
    const double* vinvT;   // np x np, [m*np + k] (transposed copy for coalesced loads)
    const int* expo;       // np x 3
    const double* coef;    // np
    int degree;
    int np;
};

__device__ __forceinline__ u64 lanemask_lt() {
    const int lane = threadIdx.x & 63;
    return (lane == 0) ? 0ull : (~0ull >> (64 - lane));
}

// LDS writes of a wave ordered before its later reads (and reads before
// later writes) without a workgroup barrier, for waves that work on their
// own data
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wave-aggregated append: every lane of the wave must call this together.
// Lanes with pred get consecutive slots of *counter; returns the slot or
// 0xffffffff for lanes without pred.
__device__ __forceinline__ u32 wave_append(u32* counter, bool pred) {
    const u64 m = __ballot(pred);
    if (m == 0) return 0xffffffffu;
    const int leader = __ffsll((unsigned long long)m) - 1;
    const int lane = threadIdx.x & 63;
    u32 base = 0;
    if (lane == leader) base = atomicAdd(counter, (u32)__popcll(m));
    base = __shfl(base, leader, 64);
    return pred ? base + (u32)__popcll(m & lanemask_lt()) : 0xffffffffu;
}

// ---- exact orientation: sign of p . (a x b) --------------------------------

__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void two_prod(double a, double b, double& p, double& e) {
    p = a * b;
    e = __fma_rn(a, b, -p);
}

// Sign of the exact value of sum_t sgn_t * x_t * y_t * z_t over six triple
// products, by error-free transformations: each triple product becomes four
// doubles summing to it exactly, and the 24 terms are accumulated into a
// non-overlapping expansion (Shewchuk's grow-expansion); the sign of the
// largest non-zero component is the sign of the sum.  Every term is appended
// (zeros included), so the expansion length at each step is a compile-time
// constant: with the loops unrolled the expansion stays in registers.
__device__ __noinline__ int orient_exact_slow(const double* a, const double* b, const double* p) {
    double e[24];
    const double tx[6] = {p[0], p[0], p[1], p[1], p[2], p[2]};
    const double ty[6] = {a[1], a[2], a[2], a[0], a[0], a[1]};
    const double tz[6] = {b[2], -b[1], b[0], -b[2], b[1], -b[0]};
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        double h1, l1, h2, l2, h3, l3;
        two_prod(tx[t], ty[t], h1, l1);
        two_prod(h1, tz[t], h2, l2);
        two_prod(l1, tz[t], h3, l3);
        const double parts[4] = {h2, l2, h3, l3};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            double q = parts[u];
            const int m = 4 * t + u;
#pragma unroll
            for (int i = 0; i < m; ++i) {
                double s, h;
                two_sum(q, e[i], s, h);
                e[i] = h;
                q = s;
            }
            e[m] = q;
        }
    }
    int sign = 0;
#pragma unroll
    for (int i = 0; i < 24; ++i) sign = e[i] > 0 ? 1 : (e[i] < 0 ? -1 : sign);
    return sign;
}

// Second stage: the determinant in double-double arithmetic.  Each 2x2
// minor a_i b_j - a_j b_i is formed from exact products (two_prod) as s + t
// with |error| <= ~4.1 eps^2 P (P the sum of the two |products|); each p_i s_i
// is an exact two_prod, each p_i t_i is rounded once, the three leading
// products are summed exactly and the eight small terms in plain FP64.  The
// total error stays below 64 eps^2 perm; the sign is taken when |det| exceeds
// twice that, otherwise -2 (undecided) is returned.
__device__ __forceinline__ int orient_dd(const double* a, const double* b, const double* p, double perm) {
#pragma clang fp contract(off)
    double hs[3], sm[8];
    int nsm = 0;
    const int i1[3] = {1, 2, 0}, i2[3] = {2, 0, 1};
    for (int c = 0; c < 3; ++c) {
        double h1, l1, h2, l2, s, e;
        two_prod(a[i1[c]], b[i2[c]], h1, l1);
        two_prod(a[i2[c]], b[i1[c]], h2, l2);
        two_sum(h1, -h2, s, e);
        const double t = (l1 - l2) + e;
        double H, Lo;
        two_prod(p[c], s, H, Lo);
        hs[c] = H;
        sm[nsm++] = Lo;
        sm[nsm++] = p[c] * t;
    }
    double A, a1, B, b1;
    two_sum(hs[0], hs[1], A, a1);
    two_sum(A, hs[2], B, b1);
    double r = a1 + b1;
    for (int i = 0; i < nsm; ++i) r += sm[i];
    const double f = B + r;
    const double eps2 = 1.2325951644078310e-32;  // 2^-106
    const double bound = 128.0 * eps2 * perm;
    if (f > bound) return 1;
    if (f < -bound) return -1;
    return -2;
}

// Bound on perm = sum_i |p_i| (|a_j b_k| + |a_k b_j|) for a and b of unit
// length (the tree's vertices, normalised in FP64): every |a_j b_k| is at
// most (1 + eps)^2, so perm <= 2 (1 + eps)^2 |p|_1.  One value per point.
__device__ __forceinline__ double perm_bound(const double* p) {
    return 2.000001 * ((fabs(p[0]) + fabs(p[1])) + fabs(p[2]));
}

// The orientation without the exact expansion: +1, -1 or 0 where the FP64
// filter, a shared vertex or the double-double stage decides, else -2.
__device__ __forceinline__ int orient_filtered(const double* a, const double* b, const double* p, double pb) {
#pragma clang fp contract(off)
    const double cx = a[1] * b[2] - a[2] * b[1];
    const double cy = a[2] * b[0] - a[0] * b[2];
    const double cz = a[0] * b[1] - a[1] * b[0];
    const double det = (p[0] * cx + p[1] * cy) + p[2] * cz;
    const double bound = 8.0 * 1.1102230246251565e-16 * pb;
    if (det > bound) return 1;
    if (det < -bound) return -1;
    // p equal to a or b: the determinant is exactly zero (grid particles are
    // the vertices of the finer triangles, so this is the common exact case)
    if ((p[0] == a[0] && p[1] == a[1] && p[2] == a[2]) || (p[0] == b[0] && p[1] == b[1] && p[2] == b[2])) return 0;
    // p the antipode of a or b (a root vertex seen from the far side)
    if ((p[0] == -a[0] && p[1] == -a[1] && p[2] == -a[2]) || (p[0] == -b[0] && p[1] == -b[1] && p[2] == -b[2]))
        return 0;
    // every term p_i (a_j b_k - a_k b_j) with a zero factor: the determinant
    // is exactly zero (a point on a root edge that lies in a coordinate plane)
    if ((p[0] == 0.0 || ((a[1] == 0.0 || b[2] == 0.0) && (a[2] == 0.0 || b[1] == 0.0))) &&
        (p[1] == 0.0 || ((a[2] == 0.0 || b[0] == 0.0) && (a[0] == 0.0 || b[2] == 0.0))) &&
        (p[2] == 0.0 || ((a[0] == 0.0 || b[1] == 0.0) && (a[1] == 0.0 || b[0] == 0.0))))
        return 0;
    return orient_dd(a, b, p, pb);
}

// Filtered exact orientation, a and b of unit length, pb = perm_bound(p).
// The plain FP64 evaluation below has a rounding error of at most about
// 5 eps * perm <= 5 eps * pb; when |det| exceeds 8 eps * pb its sign is
// certain; otherwise the double-double stage decides, and only when that
// cannot (|det| below ~1e-30, typically an exact zero) the exact expansion
// does.  Points of a grid finer than the tree lie within rounding distance
// of tree edges, so the double-double stage is common: it is inlined.
__device__ __forceinline__ int orient(const double* a, const double* b, const double* p, double pb) {
    const int o = orient_filtered(a, b, p, pb);
    return o != -2 ? o : orient_exact_slow(a, b, p);
}

// Interpolation point m of node g (Sec. 3, interpolation in triangles):
// y = normalise((b1 v1 + b2 v2) + b3 v3); returns |b1 v1 + b2 v2 + b3 v3|.
__device__ __forceinline__ double proxy_point(const NodeGeo& g, const double* b, double* y) {
    double p[3];
    for (int c = 0; c < 3; ++c) p[c] = (b[0] * g.v[0][c] + b[1] * g.v[1][c]) + b[2] * g.v[2][c];
    const double n = sqrt((p[0] * p[0] + p[1] * p[1]) + p[2] * p[2]);
    const double inv = 1.0 / n;
    y[0] = p[0] * inv;
    y[1] = p[1] * inv;
    y[2] = p[2] * inv;
    return n;
}

__device__ __forceinline__ double ipow(double x, int e) {
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

// FP64 reciprocal: hardware estimate refined by two Newton steps.
__device__ __forceinline__ double rcp64(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = __fma_rn(-d, r, 1.0);
    r = __fma_rn(r, e, r);
    e = __fma_rn(-d, r, 1.0);
    r = __fma_rn(r, e, r);
    return r;
}

__device__ __forceinline__ int level_of_offset_table(const i64* off, int L, i64 id) {
    int l = 0;
    while (l < L && off[l + 1] <= id) ++l;
    return l;
}

// q = a / b and r = a - q b for 0 <= a < 2^22, 1 <= b < 2^22: the FP32
// estimate a * rcp(b) is within 1 of the quotient (relative error below
// 2^-22), so truncating it and correcting once with the remainder is exact;
// the integer division sequence it replaces is about 30 instructions
__device__ __forceinline__ int div_small(int a, int b, int& r) {
    int q = (int)((float)a * __builtin_amdgcn_rcpf((float)b));
    r = a - q * b;
    if (r < 0) {
        --q;
        r += b;
    } else if (r >= b) {
        ++q;
        r -= b;
    }
    return q;
}

// Block-wide product out[k][c] = sum_m Mt[m * nout + k] * sc[m] * in[m][c]
// for k < nout, m < nin, c < NC, with all NT threads: thread t handles row
// k = t % nout and the m-range of group t / nout (NT / nout groups);
// partial sums meet in red (LDS, >= NT * NC doubles).  Mt is read row by
// row, consecutive threads reading consecutive k (coalesced).  sc may be
// null (all ones).  Must be called by every thread of the block; ends with a
// barrier.
template <int NT, int NC>
__device__ __forceinline__ void block_matvec(const double* __restrict__ Mt, int nin, int nout, const double* sc,
                                             const double (*in)[NC], double* red, double (*out)[NC]) {
    const int tid = threadIdx.x;
    int rem, k;
    const int G = div_small(NT, nout, rem);
    const int g = div_small(tid, nout, k);
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    if (g < G) {
        const int per = div_small(nin + G - 1, G, rem);
        const int m0 = g * per, m1 = (m0 + per) < nin ? (m0 + per) : nin;
#pragma unroll 4
        for (int m = m0; m < m1; ++m) {
            const double f = Mt[(size_t)m * nout + k] * (sc ? sc[m] : 1.0);
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[c] += f * in[m][c];
        }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) red[c * NT + tid] = (g < G) ? acc[c] : 0.0;
    __syncthreads();
    if (tid < nout) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double s = 0.0;
            for (int gg = 0; gg < G; ++gg) s += red[c * NT + gg * nout + tid];
            out[tid][c] = s;
        }
    }
    __syncthreads();
}

// host-side launch helpers (implemented in the .hip files)
constexpr int kSortMaxPasses = 8;
constexpr int kSortCopies = 8;  // each digit histogram kept in copies (atomics spread over addresses)
// digit histograms (2 arrays x kSortMaxPasses x kSortCopies x 256) and tile
// counters (2 x kSortMaxPasses); zero when a sort starts
constexpr int kSortHistWords = 2 * kSortMaxPasses * kSortCopies * 256;
constexpr int kSortZeroWords = kSortHistWords + 2 * kSortMaxPasses;
struct SortScratch {
    u32* zero;    // kSortZeroWords
    u64* status;  // 2 x max_tiles x 256 look-back status words
    u32* epoch;   // 2 counters, advanced by every sort
    u32* err;     // set if a look-back exceeded its spin bound
    int max_tiles;
};

// up to two independent key arrays sorted in the same passes
struct SortBatch {
    const u64* in[2];
    u64* out[2];
    const u32* dn[2];
};

void radix_sort(hipStream_t s, u64* keys, u64* tmp, const u32* d_n, u32 n_bound, int bit_lo,
                int bit_hi, SortScratch scratch, u64** result);
void radix_sort_batch(hipStream_t s, int nb, u64* const* keys, u64* const* tmp, const u32* const* d_n, u32 n_bound,
                      int bit_lo, int bit_hi, SortScratch scratch, u64** result);

}  // namespace stc
