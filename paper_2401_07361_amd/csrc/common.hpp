// Shared device helpers and internal declarations of the HIP library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "geometry.hpp"

namespace stc {

using u32 = uint32_t;
using u64 = uint64_t;
using i32 = int32_t;
using i64 = int64_t;

constexpr double kInv4Pi = 0.07957747154594767;  // 1 / (4 pi)
constexpr int kMaxDegree = 14;
constexpr int kMaxNp = (kMaxDegree + 1) * (kMaxDegree + 2) / 2;  // 120

// counter slots in the context's u32 counter array
enum Counter : int {
    C_TLIST = 0,      // entries in the target-particle list (PP + PC)
    C_NLIST = 1,      // entries in the target-proxy list (CP + CC)
    C_PP = 2, C_PC = 3, C_CP = 4, C_CC = 5,
    C_OVERFLOW = 6,   // set to 1 when any list or frontier outgrows capacity
    C_FRONT = 16,     // C_FRONT + k: frontier length at traversal iteration k
    C_COUNT = 64
};

// Interpolation tables on the device.
struct RefDev {
    const double* points;  // np x 3
    const double* vinv;    // np x np, [k*np + m]
    const int* expo;       // np x 3
    const double* coef;    // np
    int degree;
    int np;
};

__device__ __forceinline__ u64 lanemask_lt() {
    const int lane = threadIdx.x & 63;
    return (lane == 0) ? 0ull : (~0ull >> (64 - lane));
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
// largest non-zero component is the sign of the sum.
__device__ __noinline__ int orient_exact_slow(const double* a, const double* b, const double* p) {
    double e[24];
    int m = 0;
    const double tx[6] = {p[0], p[0], p[1], p[1], p[2], p[2]};
    const double ty[6] = {a[1], a[2], a[2], a[0], a[0], a[1]};
    const double tz[6] = {b[2], b[1], b[0], b[2], b[1], b[0]};
    const double sg[6] = {1.0, -1.0, 1.0, -1.0, 1.0, -1.0};
    for (int t = 0; t < 6; ++t) {
        double h1, l1, h2, l2, h3, l3;
        two_prod(tx[t], ty[t], h1, l1);
        two_prod(h1, sg[t] * tz[t], h2, l2);
        two_prod(l1, sg[t] * tz[t], h3, l3);
        const double parts[4] = {h2, l2, h3, l3};
        for (int u = 0; u < 4; ++u) {
            double q = parts[u];
            for (int i = 0; i < m; ++i) {
                double s, h;
                two_sum(q, e[i], s, h);
                e[i] = h;
                q = s;
            }
            e[m++] = q;
        }
    }
    for (int i = m - 1; i >= 0; --i) {
        if (e[i] > 0) return 1;
        if (e[i] < 0) return -1;
    }
    return 0;
}

// Filtered exact orientation.  The plain FP64 evaluation below has a
// rounding error of at most about 5 eps * perm; when |det| exceeds 8 eps *
// perm its sign is certain, otherwise the exact path decides.
__device__ __forceinline__ int orient(const double* a, const double* b, const double* p) {
#pragma clang fp contract(off)
    const double cx = a[1] * b[2] - a[2] * b[1];
    const double cy = a[2] * b[0] - a[0] * b[2];
    const double cz = a[0] * b[1] - a[1] * b[0];
    const double det = (p[0] * cx + p[1] * cy) + p[2] * cz;
    const double perm = fabs(p[0]) * (fabs(a[1] * b[2]) + fabs(a[2] * b[1])) +
                        fabs(p[1]) * (fabs(a[2] * b[0]) + fabs(a[0] * b[2])) +
                        fabs(p[2]) * (fabs(a[0] * b[1]) + fabs(a[1] * b[0]));
    const double bound = 8.0 * 1.1102230246251565e-16 * perm;
    if (det > bound) return 1;
    if (det < -bound) return -1;
    return orient_exact_slow(a, b, p);
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

// host-side launch helpers (implemented in the .hip files)
struct SortScratch {
    u32* hist;       // 256 * max_blocks
    int max_blocks;
};

void radix_sort(hipStream_t s, u64* keys, u64* tmp, const u32* d_n, u32 n_bound, int bit_lo,
                int bit_hi, SortScratch scratch, u64** result);

}  // namespace stc
