// Interaction kernels of the tree code (Sec. 3, treatment of clusters) and
// the direct sum (Sec. 2, discrete system).
//
// Every interaction adds  q_j (y_j - x) / den(x, y_j)  for sources y_j with
// charges q_j to a target point x: particles or proxy points on either side.
// The velocity is taken at the end as u_i = -(1/4pi) x_i x W_i, which equals
// the paper's sum because x_i x x_i = 0.
//
//  * k_near          targets = particles of a leaf:  PP (source particles)
//                    and PC (source proxy points with proxy charges).
//  * k_far_targets   targets = proxy points of a node: CP and CC; the values
//                    at the target points are turned into interpolation
//                    coefficients alpha_k = sum_n (V^{-1})_{kn} W(x~_n).
//  * k_l2p_finalize  W_i += sum_k B_k(b(x_i)) alpha_k for every node holding
//                    i that received CP/CC work; then the cross product and
//                    the scatter back to input order.
//
// Segment kernels run NTT threads per workgroup (256 by default; 128 or 512
// when the launch autotuner picks them).  A persistent grid splits
// the target-sorted list into equal contiguous ranges of entries; a
// workgroup handles every target whose run of entries starts inside its
// range.  The block -> range map is XCD aware (consecutive ranges, i.e.
// neighbouring triangles that share sources, run on the same XCD and its
// L2).  Sources are staged into NTT-entry LDS tiles, one source per thread;
// threads split as (target, source slice) with NTT / n_targets slices.
// FP32 mode: coordinates relative to the target triangle's circumcentre,
// rounded from FP64; partial sums per tile in FP32, added into FP64.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"
#include "stc.h"

namespace stc {

namespace {

template <typename T>
struct Src {
    T x, y, z, q;
};

typedef float mf32x4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ T rcp_t(T v);
template <>
__device__ __forceinline__ float rcp_t<float>(float v) {
    return __builtin_amdgcn_rcpf(v);
}
template <>
__device__ __forceinline__ double rcp_t<double>(double v) {
    return rcp64(v);
}

// A target coordinate as a value computed in a register (the FP32 rounding,
// or an FMA by 1 in FP64) rather than the register a memory load filled:
// the compiler's wait counting otherwise makes the interaction loops wait on
// every outstanding load (the next tile's) when they read such a register.
template <typename T>
__device__ __forceinline__ T target_reg(double v);
template <>
__device__ __forceinline__ float target_reg<float>(double v) {
    return (float)v;
}
template <>
__device__ __forceinline__ double target_reg<double>(double v) {
    return __fma_rn(v, 1.0, 0.0);
}

template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c) {
    return __builtin_fma(a, b, c);
}
template <>
__device__ __forceinline__ float fma_t<float>(float a, float b, float c) {
    return __builtin_fmaf(a, b, c);
}

// Stream-function kernels (Sec. 2, stream function and Green's function):
// kernel codes beside the two velocity denominators.  Their interaction adds
// q log(den) to the first component only (den = 1 - x.y, or |x - y|^2 / 2
// with the factor 1/2 applied here: the charges are not scaled), and the
// result is psi = W_0 / 4 pi.
constexpr int DEN_LOG_DOT = 2, DEN_LOG_DIST2 = 3;

template <typename T>
__device__ __forceinline__ T log_t(T v);
// FP32: the hardware base-2 logarithm (v_log_f32); the factor ln 2 that
// turns it into the natural logarithm travels with the staged charges
// (charge_scale).  The denominators here are normal numbers (|x - y|^2 / 2
// between ~1e-6 and 2 in target-relative coordinates), where the instruction
// is accurate to about one ulp; the library logf adds range reduction and
// special-case handling that cost about ten more instructions per evaluation.
template <>
__device__ __forceinline__ float log_t<float>(float v) {
    return __builtin_amdgcn_logf(v);
}
template <>
__device__ __forceinline__ double log_t<double>(double v) {
    return log(v);
}

// Factor applied to every charge as it is staged: 2 for the velocity with
// |x - y|^2 (the kernel drops the 1/2 of |x - y|^2 / 2), ln 2 for the FP32
// logarithmic kernel (its logarithm is base 2), else 1.
template <typename T, int DEN>
__device__ __forceinline__ double charge_scale() {
    if constexpr (DEN == STC_DEN_DIST2) return 2.0;
    else if constexpr (DEN >= DEN_LOG_DOT && sizeof(T) == 4) return 0.693147180559945309;
    else return 1.0;
}

// one kernel evaluation: q (y - x) / den added to (px, py, pz), or, for the
// stream function, q log(den) added to px
template <typename T, int DEN>
__device__ __forceinline__ void interact(const Src<T>& s, T tx, T ty, T tz, T& px, T& py, T& pz) {
    const T dx = s.x - tx, dy = s.y - ty, dz = s.z - tz;
    if constexpr (DEN >= DEN_LOG_DOT) {
        T den;
        if constexpr (DEN == DEN_LOG_DIST2) den = T(0.5) * (dx * dx + dy * dy + dz * dz);
        else den = fma_t<T>(-tx, s.x, fma_t<T>(-ty, s.y, fma_t<T>(-tz, s.z, T(1))));
        px += s.q * log_t<T>(den);
    } else {
        T den;
        if (DEN == STC_DEN_DIST2) den = dx * dx + dy * dy + dz * dz;  // charges carry the factor 2
        else den = fma_t<T>(-tx, s.x, fma_t<T>(-ty, s.y, fma_t<T>(-tz, s.z, T(1))));  // 1 - x.y in three FMAs
        const T w = s.q * rcp_t<T>(den);
        px += w * dx;
        py += w * dy;
        pz += w * dz;
    }
}

// Four FP64 kernel evaluations with one reciprocal: v_rcp_f64 issues at a
// quarter of the FMA rate and needs two Newton steps, so 1 / (d0 d1 d2 d3)
// is formed once and each 1 / d_k recovered by multiplying it with the other
// three denominators (a few ulp, against the half ulp of four separate
// reciprocals).  The denominators lie in (0, 2] and above ~1e-20 for any
// two distinct points a double can tell apart near the sphere, so the
// product neither overflows nor underflows; a zero denominator (coincident
// particles) makes all four non-finite, as it makes its own one with
// separate reciprocals.
template <int DEN>
__device__ __forceinline__ void interact4(const Src<double>* __restrict__ s, double tx, double ty, double tz,
                                          double& px, double& py, double& pz) {
    if constexpr (DEN >= DEN_LOG_DOT) {  // no reciprocal to share
#pragma unroll
        for (int k = 0; k < 4; ++k) interact<double, DEN>(s[k], tx, ty, tz, px, py, pz);
        return;
    }
    double dx[4], dy[4], dz[4], den[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        dx[k] = s[k].x - tx, dy[k] = s[k].y - ty, dz[k] = s[k].z - tz;
        if (DEN == STC_DEN_DIST2) den[k] = dx[k] * dx[k] + dy[k] * dy[k] + dz[k] * dz[k];
        else den[k] = __fma_rn(-tx, s[k].x, __fma_rn(-ty, s[k].y, __fma_rn(-tz, s[k].z, 1.0)));
    }
    const double p01 = den[0] * den[1], p23 = den[2] * den[3];
    const double r = rcp64(p01 * p23);
    const double r01 = r * p23, r23 = r * p01;  // 1 / (d0 d1), 1 / (d2 d3)
    const double inv[4] = {r01 * den[1], r01 * den[0], r23 * den[3], r23 * den[2]};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double w = s[k].q * inv[k];
        px += w * dx[k];
        py += w * dy[k];
        pz += w * dz[k];
    }
}

// Sum over this slice's staged sources for the thread's TP targets (each
// source read from LDS once and used for all of them): slice sl takes the
// contiguous block [sl m, (sl + 1) m) of the tile, m = cnt / S (the same trip
// count in every lane, so the loop unrolls with constant LDS offsets from one
// base), then at most one of the cnt - S m remaining sources, S m + sl.  With
// SELF, source self_j[k] is skipped for target k (the j = i exclusion).
template <typename T, int DEN, bool SELF, int TP>
__device__ __forceinline__ void tile_sum(const Src<T>* __restrict__ tile, int cnt, int sl, int S, const T* tx,
                                         const T* ty, const T* tz, const int* self_j, double* ax, double* ay,
                                         double* az) {
    T px[TP], py[TP], pz[TP];
#pragma unroll
    for (int k = 0; k < TP; ++k) px[k] = py[k] = pz[k] = T(0);
    if (!SELF) {
        int mr;
        const int m = div_small(cnt, S, mr);
        const Src<T>* __restrict__ blk = tile + sl * m;
        if constexpr (sizeof(T) == 8) {
            int it = 0;
            for (; it + 4 <= m; it += 4) {
                Src<T> src[4];
#pragma unroll
                for (int l = 0; l < 4; ++l) src[l] = blk[it + l];
#pragma unroll
                for (int k = 0; k < TP; ++k) interact4<DEN>(src, tx[k], ty[k], tz[k], px[k], py[k], pz[k]);
            }
            for (; it < m; ++it) {
                const Src<T> src = blk[it];
#pragma unroll
                for (int k = 0; k < TP; ++k) interact<T, DEN>(src, tx[k], ty[k], tz[k], px[k], py[k], pz[k]);
            }
        } else {
#pragma unroll 4
            for (int it = 0; it < m; ++it) {
                const Src<T> src = blk[it];
#pragma unroll
                for (int k = 0; k < TP; ++k) interact<T, DEN>(src, tx[k], ty[k], tz[k], px[k], py[k], pz[k]);
            }
        }
        const int j = S * m + sl;
        if (j < cnt) {
            const Src<T> src = tile[j];
#pragma unroll
            for (int k = 0; k < TP; ++k) interact<T, DEN>(src, tx[k], ty[k], tz[k], px[k], py[k], pz[k]);
        }
    } else {
        for (int j = sl; j < cnt; j += S) {
            const Src<T> src = tile[j];
#pragma unroll
            for (int k = 0; k < TP; ++k)
                if (j != self_j[k]) interact<T, DEN>(src, tx[k], ty[k], tz[k], px[k], py[k], pz[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < TP; ++k) {
        ax[k] += (double)px[k];
        ay[k] += (double)py[k];
        az[k] += (double)pz[k];
    }
}

__device__ __forceinline__ u32 logical_block() {
    const u32 G = gridDim.x, b = blockIdx.x;
    return (b % 8u) * (G / 8u) + (b / 8u);
}

// Position in the list of workgroup b of a segment kernel.  The dispatcher
// deals workgroups to the eight XCDs in turn (b runs on XCD b % 8); each XCD
// takes runs of kXcdRun consecutive list chunks, the runs dealt to the XCDs
// in turn, so that neighbouring chunks (which share sources) meet in one L2
// while every XCD gets its share of each part of the list.  (Contiguous
// eighths of the list per XCD, as logical_block gives, put the coarse levels'
// target nodes, which come first and can carry several times the work of the
// fine ones, on one XCD: 2.2 times the mean work there on the learned form's
// far list at N = 2621442.)  A bijection of [0, G) for G a multiple of 8.
constexpr u32 kXcdRun = 16;
__device__ __forceinline__ u32 segment_block() {
    const u32 G = gridDim.x, b = blockIdx.x;
    if (G % 8u) return b;
    const u32 q = b / 8u, x = b % 8u, Q = q / kXcdRun, j = q % kXcdRun;
    const u32 full = (G / 8u) / kXcdRun;  // complete runs per XCD
    const u32 run = Q < full ? kXcdRun : (G / 8u) - full * kXcdRun;
    return Q * 8u * kXcdRun + x * run + j;
}

// Matrix-core form of the FP32 velocity kernel of the target proxies
// (k_far_targets, |x - y|^2 denominator).  For a group of 16 target points x
// and a chunk of 16 sources y (both relative to the target node's centre)
// the denominators form a rank-4 product plus a rank-1 term,
//   |x - y|^2 = |x|^2 + (y, |y|^2) . (-2 x, 1),
// one v_mfma_f32_16x16x4f32 with the sources as A (16 x 4), the targets as
// B (4 x 16) and |x|^2 as C; the VALU takes the reciprocals of the 256
// results; four v_mfma_f32_4x4x1f32 then add r times the rows q (y, 1) into
// 4 x 4 blocks (block b: targets 4 (b % 4) .. + 3, sources 4 (b / 4) + i of
// the chunk in step i), so that
//   W(x) = sum_j r q_j y_j - x sum_j r q_j
// is recovered from the blocks' four columns.  The VALU issues one reciprocal
// per pair instead of eleven instructions.  Both rewrites cost accuracy where
// |y| (target-relative) is much larger than |y - x|: FP32 rounding grows by
// about (|x| + |y|)^2 / |x - y|^2 in the denominator and |y| / |y - x| in the
// sum; for CP and CC pairs the acceptance criterion bounds both ratios
// ((1 + theta) / (1 - theta) for the second, its square for the first); for
// near-field pairs they are unbounded, so k_near keeps the VALU form.
// Operand layouts (measured): 16x16x4 A[i][k] in lane 16 k + i, B[k][j] in
// lane 16 k + j, D[i][j] in lane 16 (i / 4) + j register i % 4; 4x4x1 block b
// row i from lane 4 b + i (A), column j from lane 4 b + j (B), D[b][i][j] in
// lane 4 b + j register i.  Up to 80 target points per pass (5 groups,
// degree <= 11).
// Measured issue costs on gfx950 (cycles per wave instruction per SIMD):
// FP32 FMA 4, v_rcp_f32 8, 16x16x4 MFMA 32, 4x4x1 MFMA 8.  Per 256 pairs
// this form needs 64 matrix-core and 32 VALU cycles against 192 VALU cycles,
// but within one wave each chunk is a dependent chain (MFMA -> reciprocal ->
// MFMA) and the kernel reaches about a third of that bound: on gv_l8
// (theta 0.8, d 10) 0.400 ms against 0.375 ms for the VALU form (both with
// k_far_finish), E 5.01e-7 against 4.95e-7.  The library is built with the
// VALU form; -DSTC_FAR_MFMA=1 (environment STC_FAR_MFMA=1 for the build
// script) selects this one.
#ifndef STC_FAR_MFMA
#define STC_FAR_MFMA 0
#endif
constexpr int kMfTargets = 80;
constexpr int kMfGroups = kMfTargets / 16;

// LDS of a segment kernel with NTT threads: one tile of 2 NTT sources (two
// consecutive ones staged per thread), one batch of NTT list entries, and
// the per-slice partial sums, which share the tiles' space (they are
// written after the last tile is used).  The matrix-core form (MF) stages
// each source's (x, y, z, 1) transposed per chunk of 16 ([chunk][c][l % 16],
// so that the A operand's lanes read consecutive words), its |y|^2, and its
// row q (y, 1), the rows of four consecutive sources interleaved by
// component ([(l / 4) 4 + c][l % 4]) so that a lane reads its four B
// operands with one 16-byte load; its partial sums are per wave, and the
// pass's target points (x, |x|^2) sit in tgt.
// (The matrix-core members are empty placeholders in the VALU form, so that
// its layout, and with it the kernels' register allocation, is unchanged.)
template <int NTT, bool MF>
struct MfShared {
    struct Tiles {
        float y[2 * NTT / 16][4][16];  // per chunk of 16 sources: x, y, z, 1 (the A operand's rows)
        mf32x4 row[2 * NTT];  // q (x, y, z, 1), four sources interleaved by component
        float b[2 * NTT];     // |y|^2
    };
    struct Sums {
        double v[NTT / 64][kMfTargets][4];  // per-wave sums (columns q y, q) of the pass's targets
    };
    struct Targets {
        mf32x4 v[kMfTargets];  // the pass's target points (x, |x|^2)
    };
};
template <int NTT>
struct MfShared<NTT, false> {
    struct Tiles {
        float unused;
    };
    using Sums = Tiles;
    using Targets = Tiles;
};

template <typename T, int NTT, int TP, bool MF>
struct SegShared {
    struct Tiles {
        Src<T> tile[2 * NTT];
    };
    union {
        Tiles t;
        typename MfShared<NTT, MF>::Tiles m;
        double red[TP][3][NTT];  // per-slice partial sums of each thread's TP targets
        typename MfShared<NTT, MF>::Sums wred;
    } u;
    u32 ent_s[NTT];        // source node of a particle entry, storage slot of a proxy entry
    i32 ent_first[NTT];    // first particle of a particle source, -1 for proxy points
    u32 ent_pre[NTT + 1];  // exclusive prefix of the entries' source counts
    u32 wave_tot[NTT / 64];
    int self_flag;
    typename MfShared<NTT, MF>::Targets tgt;
};

// exclusive prefix over the NTT threads; returns the prefix, *total the sum
template <int NTT>
__device__ __forceinline__ u32 block_exclusive_scan(u32 v, u32* wave_tot, u32* total) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    u32 incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        const u32 t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) wave_tot[w] = incl;
    __syncthreads();
    u32 base = 0, tot = 0;
    for (int k = 0; k < NTT / 64; ++k) {
        const u32 wt = wave_tot[k];
        if (k < w) base += wt;
        tot += wt;
    }
    *total = tot;
    return base + incl - v;
}

// One source point relative to (cx, cy, cz), charge scaled by qscale: point l
// of particle range `first`, or (first < 0) proxy record s + l (s: first
// record of the source node's degree class).
template <typename T>
__device__ __forceinline__ Src<T> load_source(const EvalArgs& a, u32 s, i32 first, int l, double cx, double cy,
                                              double cz, double qscale) {
    Src<T> v;
    if (first >= 0) {
        const i32 j = first + l;
        v.x = (T)(a.sx[j] - cx);
        v.y = (T)(a.sy[j] - cy);
        v.z = (T)(a.sz[j] - cz);
        v.q = (T)(qscale * a.sq[j]);
    } else {
        const Prox pr = a.prox[(size_t)s + l];
        v.x = (T)(pr.x - cx);
        v.y = (T)(pr.y - cy);
        v.z = (T)(pr.z - cz);
        v.q = (T)(qscale * pr.w);
    }
    return v;
}

// Writes source v to tile slot l.
template <typename T, int NTT, int TP>
__device__ __forceinline__ void stage(SegShared<T, NTT, TP, false>& sh, int l, const Src<T>& v) {
    sh.u.t.tile[l] = v;
}

// Matrix-core form: source v (or, with dummy, a source of charge zero at the
// origin with |y|^2 = 1, which pads a chunk to 16) to slot l.
template <int NTT, int TP>
__device__ __forceinline__ void stage_mf(SegShared<float, NTT, TP, true>& sh, int l, const Src<float>& v, bool dummy) {
    float* row = reinterpret_cast<float*>(sh.u.m.row) + (((l >> 2) * 4) << 2) + (l & 3);
    if (dummy) {
        sh.u.m.y[l >> 4][0][l & 15] = 0.f;
        sh.u.m.y[l >> 4][1][l & 15] = 0.f;
        sh.u.m.y[l >> 4][2][l & 15] = 0.f;
        sh.u.m.y[l >> 4][3][l & 15] = 1.f;
        sh.u.m.b[l] = 1.f;
        row[0] = row[4] = row[8] = row[12] = 0.f;
        return;
    }
    const double b = ((double)v.x * v.x + (double)v.y * v.y) + (double)v.z * v.z;
    sh.u.m.y[l >> 4][0][l & 15] = v.x;
    sh.u.m.y[l >> 4][1][l & 15] = v.y;
    sh.u.m.y[l >> 4][2][l & 15] = v.z;
    sh.u.m.y[l >> 4][3][l & 15] = 1.f;
    sh.u.m.b[l] = (float)b;
    row[0] = v.q * v.x;
    row[4] = v.q * v.y;
    row[8] = v.q * v.z;
    row[12] = v.q;
}

template <typename T, int DEN, bool SELF, int TP>
__device__ __forceinline__ void tile_sum_acc(const Src<T>* __restrict__ tile, int cnt, int sl, int S, const T* tx,
                                             const T* ty, const T* tz, const int* self_j, double (*acc)[4]) {
    double ax[TP], ay[TP], az[TP];
#pragma unroll
    for (int k = 0; k < TP; ++k) ax[k] = acc[k][0], ay[k] = acc[k][1], az[k] = acc[k][2];
    tile_sum<T, DEN, SELF, TP>(tile, cnt, sl, S, tx, ty, tz, self_j, ax, ay, az);
#pragma unroll
    for (int k = 0; k < TP; ++k) acc[k][0] = ax[k], acc[k][1] = ay[k], acc[k][2] = az[k];
}

// Accumulates, for this thread's TP targets, every entry of [e0, e1) in
// `list` whose type bit is in type_mask.  Entries are taken in batches of
// NTT: their source counts are scanned into an LDS prefix, so that for each
// NTT-source tile every thread stages exactly one source (its entry found by
// binary search) and all global loads of a tile are in flight together.  A
// PP entry whose source is the target leaf itself (self_t) is evaluated on
// its own with the j != i exclusion (me: the targets' indices there).
// acc[k]: the target's sums (x, y, z).
template <typename T, int DEN, int NTT, int TP>
__device__ void accumulate_entries(const EvalArgs& a, const u64* __restrict__ list, u32 e0, u32 e1, u32 type_mask,
                                   u32 self_t, const int* me, bool act, int sl, int S, const T* tx, const T* ty,
                                   const T* tz, double cx, double cy, double cz, SegShared<T, NTT, TP, false>& sh,
                                   double (*acc)[4]) {
    const int tid = threadIdx.x;
    const u64 mask = ((u64)1 << a.W) - 1;
    const u32 cmask = (1u << a.DB) - 1u;
    const double qscale = charge_scale<T, DEN>();
    for (u32 eb = e0; eb < e1; eb += NTT) {
        const u32 ne = (e1 - eb) < (u32)NTT ? (e1 - eb) : (u32)NTT;
        if (tid == 0) sh.self_flag = 0;
        __syncthreads();
        u32 size = 0;
        if ((u32)tid < ne) {
            const u64 key = list[eb + tid];
            const int type = (int)((key >> a.W) & 1u);
            const u32 s = (u32)(key & mask);
            sh.ent_s[tid] = s;
            if ((type_mask >> type) & 1u) {
                if (type == 0) {
                    const i32 b = a.nbeg[s];
                    sh.ent_first[tid] = b;
                    if (s == self_t) sh.self_flag = 1;
                    else size = (u32)(a.nend[s] - b);
                } else {
                    const int c = (int)((key >> (a.W + 1)) & cmask);
                    sh.ent_s[tid] = (u32)a.slot[s] * (u32)a.NPT + (u32)STC_PICK4(a.cls.poff, c);
                    sh.ent_first[tid] = -1;
                    size = (u32)STC_PICK4(a.cls.np, c);
                }
            } else {
                sh.ent_first[tid] = 0;
            }
        }
        u32 total = 0;
        const u32 pre = block_exclusive_scan<NTT>(size, sh.wave_tot, &total);
        if ((u32)tid < ne) sh.ent_pre[tid] = pre;
        if (tid == 0) sh.ent_pre[ne] = total;
        __syncthreads();
        if (sh.self_flag) {
            const i32 tb = a.nbeg[self_t];
            const int nsrc = a.nend[self_t] - tb;
            for (int j0 = 0; j0 < nsrc; j0 += 2 * NTT) {
                const int cnt = (nsrc - j0) < 2 * NTT ? (nsrc - j0) : 2 * NTT;
                for (int l = tid; l < cnt; l += NTT) stage(sh, l, load_source<T>(a, self_t, tb, j0 + l, cx, cy, cz, qscale));
                __syncthreads();
                int sj[TP];
#pragma unroll
                for (int k = 0; k < TP; ++k) sj[k] = me[k] - j0;
                if (act) tile_sum_acc<T, DEN, true, TP>(sh.u.t.tile, cnt, sl, S, tx, ty, tz, sj, acc);
                __syncthreads();
            }
        }
        for (u32 g0 = 0; g0 < total; g0 += 2 * NTT) {
            const int cnt = (total - g0) < (u32)(2 * NTT) ? (int)(total - g0) : 2 * NTT;
            const int l0 = 2 * tid;
            if (l0 < cnt) {
                // the entry holding source g: binary search over the prefix;
                // source g + 1 lies in the same entry or a later one
                const u32 g = g0 + l0;
                u32 lo = 0, hi = ne;
                while (hi - lo > 1) {
                    const u32 mid = (lo + hi) >> 1;
                    if (sh.ent_pre[mid] <= g) lo = mid;
                    else hi = mid;
                }
                stage(sh, l0, load_source<T>(a, sh.ent_s[lo], sh.ent_first[lo], (int)(g - sh.ent_pre[lo]), cx, cy, cz,
                                             qscale));
                if (l0 + 1 < cnt) {
                    while (sh.ent_pre[lo + 1] <= g + 1) ++lo;  // ent_pre[ne] = total > g + 1
                    stage(sh, l0 + 1, load_source<T>(a, sh.ent_s[lo], sh.ent_first[lo], (int)(g + 1 - sh.ent_pre[lo]),
                                                     cx, cy, cz, qscale));
                }
            }
            __syncthreads();
            if (act) tile_sum_acc<T, DEN, false, TP>(sh.u.t.tile, cnt, sl, S, tx, ty, tz, nullptr, acc);
            __syncthreads();
        }
    }
}

// Matrix-core form of one tile: wave w takes the 16-source chunks w, w + NW,
// ... of the cntp (a multiple of 16) staged sources; for each of the NG
// target groups, one 16x16x4 product (A: the sources (y, 1), B: the group's
// (-2 x, |x|^2), C: the sources' |y|^2) gives the 256 denominators, the VALU
// their reciprocals, and four 4x4x1 products add r q (y, 1) into the
// group's blocks (acc[g]); the groups' products are independent, so their
// latencies overlap.  bop[g]: this lane's B operand of group g.
template <int NG, int NTT, int TP>
__device__ __forceinline__ void tile_sum_mfma(const SegShared<float, NTT, TP, true>& sh, int cntp, const float* bop,
                                              mf32x4* acc) {
    constexpr int NW = NTT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const float* __restrict__ yf = &sh.u.m.y[0][0][0];
    const mf32x4* __restrict__ bq = reinterpret_cast<const mf32x4*>(sh.u.m.b);
    for (int ch = w; ch * 16 < cntp; ch += NW) {
        const float ya = yf[ch * 64 + lane];  // A[lane % 16][lane / 16]: consecutive lanes, no bank conflicts
        const mf32x4 b = sh.u.m.row[(ch * 4 + (lane >> 4)) * 4 + (lane & 3)];
        const mf32x4 c = bq[ch * 4 + (lane >> 4)];  // |y|^2 of rows 4 (lane / 16) + i
        mf32x4 den[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) den[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(ya, bop[g], c, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int g = 0; g < NG; ++g)
                acc[g] = __builtin_amdgcn_mfma_f32_4x4x1f32(__builtin_amdgcn_rcpf(den[g][i]), b[i], acc[g], 0, 0, 0);
    }
}

// accumulate_entries for the matrix-core form (target proxies; no self
// pair): the same entry batches and tiles, sources staged as y, |y|^2 and
// rows, each tile padded to a multiple of 16 by sources of charge zero.  The
// block sums stay in FP32 over the pass (acc, per lane: about a quarter of
// the pass's sources per accumulator).
template <int NG, int NTT, int TP>
__device__ void accumulate_entries_mf(const EvalArgs& a, const u64* __restrict__ list, u32 e0, u32 e1, double cx,
                                      double cy, double cz, SegShared<float, NTT, TP, true>& sh, const float* bop,
                                      mf32x4* acc) {
    const int tid = threadIdx.x;
    const u64 mask = ((u64)1 << a.W) - 1;
    const u32 cmask = (1u << a.DB) - 1u;
    const double qscale = charge_scale<float, STC_DEN_DIST2>();
    for (u32 eb = e0; eb < e1; eb += NTT) {
        const u32 ne = (e1 - eb) < (u32)NTT ? (e1 - eb) : (u32)NTT;
        u32 size = 0;
        if ((u32)tid < ne) {
            const u64 key = list[eb + tid];
            const int type = (int)((key >> a.W) & 1u);
            const u32 s = (u32)(key & mask);
            if (type == 0) {
                const i32 b = a.nbeg[s];
                sh.ent_s[tid] = s;
                sh.ent_first[tid] = b;
                size = (u32)(a.nend[s] - b);
            } else {
                const int c = (int)((key >> (a.W + 1)) & cmask);
                sh.ent_s[tid] = (u32)a.slot[s] * (u32)a.NPT + (u32)STC_PICK4(a.cls.poff, c);
                sh.ent_first[tid] = -1;
                size = (u32)STC_PICK4(a.cls.np, c);
            }
        }
        u32 total = 0;
        const u32 pre = block_exclusive_scan<NTT>(size, sh.wave_tot, &total);
        if ((u32)tid < ne) sh.ent_pre[tid] = pre;
        if (tid == 0) sh.ent_pre[ne] = total;
        __syncthreads();
        for (u32 g0 = 0; g0 < total; g0 += 2 * NTT) {
            const int cnt = (total - g0) < (u32)(2 * NTT) ? (int)(total - g0) : 2 * NTT;
            const int cntp = (cnt + 15) & ~15;
            const int l0 = 2 * tid;
            if (l0 < cnt) {
                // the entry holding source g: binary search over the prefix;
                // source g + 1 lies in the same entry or a later one
                const u32 g = g0 + l0;
                u32 lo = 0, hi = ne;
                while (hi - lo > 1) {
                    const u32 mid = (lo + hi) >> 1;
                    if (sh.ent_pre[mid] <= g) lo = mid;
                    else hi = mid;
                }
                stage_mf(sh, l0, load_source<float>(a, sh.ent_s[lo], sh.ent_first[lo], (int)(g - sh.ent_pre[lo]), cx,
                                                    cy, cz, qscale), false);
                if (l0 + 1 < cnt) {
                    while (sh.ent_pre[lo + 1] <= g + 1) ++lo;  // ent_pre[ne] = total > g + 1
                    stage_mf(sh, l0 + 1, load_source<float>(a, sh.ent_s[lo], sh.ent_first[lo],
                                                            (int)(g + 1 - sh.ent_pre[lo]), cx, cy, cz, qscale), false);
                } else if (l0 + 1 < cntp) {
                    stage_mf(sh, l0 + 1, Src<float>{}, true);
                }
            } else if (l0 < cntp) {
                stage_mf(sh, l0, Src<float>{}, true);
                if (l0 + 1 < cntp) stage_mf(sh, l0 + 1, Src<float>{}, true);
            }
            __syncthreads();
            tile_sum_mfma<NG>(sh, cntp, bop, acc);
            __syncthreads();
        }
    }
}

// A pass over up to TP x NTT targets: thread (ti, sl) takes targets ti,
// ti + h, ... (h = ceil(ntc / TP)) and source slice sl of S = NTT / h.
// Targets past ntc duplicate a valid one and are not written back.
template <int TP>
struct TargetGroup {
    int h, S, ti, sl, me[TP];
    bool act, valid[TP];
    __device__ TargetGroup(int ntc, int nthreads, int base) {
        h = (ntc + TP - 1) / TP;
        int r;
        S = div_small(nthreads, h, r);
        sl = div_small((int)threadIdx.x, h, ti);
        act = sl < S;
#pragma unroll
        for (int k = 0; k < TP; ++k) {
            valid[k] = ti + k * h < ntc;
            me[k] = base + (valid[k] ? ti + k * h : ti);
        }
    }
};

// The sums over the S source slices of the partial sums in red (target ti +
// k h of the pass, component c, slice q at red[k][c][q h + ti]): one
// (target, component) per thread, slices added in order from zero, as a
// single thread per target would; f(target of the pass, c, sum).
template <int NTT, int TP, typename F>
__device__ __forceinline__ void slice_sums(const double (*red)[3][NTT], int h, int S, int ntc, F&& f) {
    for (int o = threadIdx.x; o < 3 * TP * h; o += NTT) {
        // o < 3 TP h: the quotients are small and come from comparisons
        int k = 0;
#pragma unroll
        for (int j = 1; j < TP; ++j) k += o >= j * 3 * h;
        const int rem = o - k * 3 * h;
        const int c = (rem >= h) + (rem >= 2 * h), ti = rem - c * h;
        if (ti + k * h < ntc) {
            double sum = 0.0;
            for (int q = 0; q < S; ++q) sum += red[k][c][q * h + ti];
            f(ti + k * h, c, sum);
        }
    }
}

// range of list entries of this workgroup (segments: key >> sh); returns
// false if empty.  spread: list chunks by segment_block (the far lists,
// whose coarse target nodes carry more work), else by logical_block (the
// near lists: target leaves of similar work, and neighbouring leaves, which
// share sources, in one XCD's L2).
template <bool SPREAD>
__device__ __forceinline__ bool wg_range(u32 n, const u64* list, const i32* seg_end, int sh, u32& e, u32& e_hi) {
    const u32 G = gridDim.x;
    const u32 chunk = (n + G - 1) / G;
    const u64 lo = (u64)(SPREAD ? segment_block() : logical_block()) * chunk;
    if (lo >= n) return false;
    e = (u32)lo;
    e_hi = (u64)e + chunk < n ? e + chunk : n;
    if (e > 0 && (list[e] >> sh) == (list[e - 1] >> sh)) e = (u32)seg_end[list[e] >> sh];
    return true;
}

constexpr int NEAR_TP = 1;  // targets per thread: leaves are small, occupancy matters more
constexpr int FAR_TP = 3;   // the proxy points of a node: each staged source feeds three targets (66 = 22 x 3: 242 of 256 threads busy, against 231 at two)

// The per-slice partial sums of a pass into LDS, three components per
// thread.
template <typename T, int NTT, int TP>
__device__ __forceinline__ void store_partials(SegShared<T, NTT, TP, false>& sh, bool act, const double (*acc)[4]) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < TP; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) sh.u.red[k][c][tid] = act ? acc[k][c] : 0.0;
}

// The learned form's far segment of one target node in a single pass over
// its entries, every degree class present at once (a pass per class would
// repeat the segment's chain of dependent loads, its barriers and its slice
// reduction for each class).  Class c with n_c sources in the segment takes
// h_c = ceil(np_c / TP) target groups times S_c slices of the workgroup's
// threads, S_c = 1 + floor((NTT - sum h) n_c / sum h n), and a region of K_c =
// floor(2 NTT S_c / sum S) slots of every tile, filled with the class's next
// K_c sources, so that every active thread sums about the same number of
// sources in every tile.  With one class this is the fixed-degree pass:
// S = floor(NTT / h), K = 2 NTT, the same staging, slices and sums.
// (Every class fits at once: np <= 120 for d <= 14, so sum h <= 108 <= NTT.)
struct LearnedSplit {
    u32 src[4];   // sources of each class in the current entry batch
    u32 tot[4];   // ... in the whole segment
    u32 bp[4];    // first source of each class in the batch's prefix
    int base[4], h[4], S[4], K[4], R[4];
    int nout[5];  // exclusive prefix of the classes' 3 TP h reduction slots
};

// Entry batch [eb, eb + ne) of a learned far segment: sources per entry and
// their prefix into sh, the batch's sources per class into sp.src / sp.bp
// (entries are sorted by class).  Starts and ends with a barrier.
template <typename T, int NTT, int TP>
__device__ void learned_batch(const EvalArgs& a, u32 eb, u32 ne, SegShared<T, NTT, TP, false>& sh, LearnedSplit& sp) {
    const int tid = threadIdx.x;
    const u64 mask = ((u64)1 << a.W) - 1;
    const u32 cmask = (1u << a.DB) - 1u;
    if (tid < 4) sp.src[tid] = 0u;
    __syncthreads();
    u32 size = 0;
    if ((u32)tid < ne) {
        const u64 key = a.nlist[eb + tid];
        const u32 s = (u32)(key & mask);
        const int c = (int)((key >> (a.W + 1)) & cmask);
        if (((key >> a.W) & 1u) == 0u) {  // CP: the particles of source node s
            const i32 b = a.nbeg[s];
            sh.ent_s[tid] = s;
            sh.ent_first[tid] = b;
            size = (u32)(a.nend[s] - b);
        } else {  // CC: the proxy points of s's class-c record
            sh.ent_s[tid] = (u32)a.slot[s] * (u32)a.NPT + (u32)STC_PICK4(a.cls.poff, c);
            sh.ent_first[tid] = -1;
            size = (u32)STC_PICK4(a.cls.np, c);
        }
        atomicAdd(&sp.src[c], size);
    }
    u32 total = 0;
    const u32 pre = block_exclusive_scan<NTT>(size, sh.wave_tot, &total);
    if ((u32)tid < ne) sh.ent_pre[tid] = pre;
    if (tid == 0) {
        sh.ent_pre[ne] = total;
        u32 p = 0;
        for (int c = 0; c < 4; ++c) {
            sp.bp[c] = p;
            p += sp.src[c];
        }
    }
    __syncthreads();
}

// W(x~_m) of every class present in target node t's learned far segment
// [e, se), written to the classes' records at rec; the classes present
// (those with sources) go to cls_mask[slot].  Ends with a barrier.
template <typename T, int DEN, int NTT, int TP>
__device__ void learned_far_values(const EvalArgs& a, u32 e, u32 se, u32 t, size_t rec, double cx, double cy,
                                   double cz, SegShared<T, NTT, TP, false>& sh) {
    __shared__ LearnedSplit sp;
    const int tid = threadIdx.x;
    const double qscale = charge_scale<T, DEN>();
    const u32 nseg = se - e;
    learned_batch(a, e, nseg < (u32)NTT ? nseg : (u32)NTT, sh, sp);
    if (tid < 4) sp.tot[tid] = sp.src[tid];
    for (u32 eb = e + NTT; eb < se; eb += NTT) {  // a segment longer than one batch: its totals first
        learned_batch(a, eb, (se - eb) < (u32)NTT ? (se - eb) : (u32)NTT, sh, sp);
        if (tid < 4) sp.tot[tid] += sp.src[tid];
    }
    __syncthreads();
    if (tid == 0) {
        int H = 0;
        u64 hw = 0;
        for (int c = 0; c < 4; ++c) {
            sp.h[c] = sp.tot[c] ? (STC_PICK4(a.cls.np, c) + TP - 1) / TP : 0;
            H += sp.h[c];
            hw += (u64)sp.h[c] * sp.tot[c];
        }
        int base = 0, sum_s = 0, no = 0;
        for (int c = 0; c < 4; ++c) {
            sp.S[c] = sp.h[c] ? 1 + (int)((u64)(NTT - H) * sp.tot[c] / hw) : 0;
            sp.base[c] = base;
            base += sp.h[c] * sp.S[c];
            sum_s += sp.S[c];
            sp.nout[c] = no;
            no += 3 * TP * sp.h[c];
        }
        sp.nout[4] = no;
        int R = 0;
        for (int c = 0; c < 4; ++c) {
            sp.K[c] = sp.S[c] ? (2 * NTT * sp.S[c]) / sum_s : 0;
            sp.R[c] = R;
            R += sp.K[c];
        }
    }
    __syncthreads();
    // this thread's class, target group ti and slice sl
    int c = -1;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (tid >= sp.base[k] && tid < sp.base[k] + sp.h[k] * sp.S[k]) c = k;
    const bool act = c >= 0;
    const int cc = act ? c : 0;
    const int h = act ? sp.h[cc] : 1;
    int ti;
    const int sl = div_small(act ? tid - sp.base[cc] : 0, h, ti);
    const int np = STC_PICK4(a.cls.np, cc);
    const Prox* __restrict__ tp = a.prox + rec + STC_PICK4(a.cls.poff, cc);
    T tx[TP], ty[TP], tz[TP];
#pragma unroll
    for (int k = 0; k < TP; ++k) {
        const int m = ti + k * h < np ? ti + k * h : ti;
        const Prox pm = tp[act ? m : 0];
        tx[k] = target_reg<T>(pm.x - cx);
        ty[k] = target_reg<T>(pm.y - cy);
        tz[k] = target_reg<T>(pm.z - cz);
    }
    double acc[TP][4];
#pragma unroll
    for (int k = 0; k < TP; ++k) acc[k][0] = acc[k][1] = acc[k][2] = acc[k][3] = 0.0;
    for (u32 eb = e; eb < se; eb += NTT) {
        const u32 ne = (se - eb) < (u32)NTT ? (se - eb) : (u32)NTT;
        if (nseg > (u32)NTT) learned_batch(a, eb, ne, sh, sp);
        int ntile = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (sp.K[k]) {
                const int nt = (int)((sp.src[k] + (u32)sp.K[k] - 1u) / (u32)sp.K[k]);
                ntile = nt > ntile ? nt : ntile;
            }
        for (int it = 0; it < ntile; ++it) {
#pragma unroll
            for (int l = 2 * tid; l < 2 * tid + 2; ++l) {
                int rc = -1;  // the class region holding tile slot l
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (l >= sp.R[k] && l < sp.R[k] + sp.K[k]) rc = k;
                if (rc < 0) continue;
                const u32 off = (u32)it * (u32)sp.K[rc] + (u32)(l - sp.R[rc]);
                if (off >= sp.src[rc]) continue;
                const u32 g = sp.bp[rc] + off;  // the entry holding batch source g
                u32 lo = 0, hi = ne;
                while (hi - lo > 1) {
                    const u32 mid = (lo + hi) >> 1;
                    if (sh.ent_pre[mid] <= g) lo = mid;
                    else hi = mid;
                }
                stage(sh, l,
                      load_source<T>(a, sh.ent_s[lo], sh.ent_first[lo], (int)(g - sh.ent_pre[lo]), cx, cy, cz, qscale));
            }
            __syncthreads();
            if (act) {
                const u32 off = (u32)it * (u32)sp.K[c];
                const int cnt = off < sp.src[c] ? ((sp.src[c] - off) < (u32)sp.K[c] ? (int)(sp.src[c] - off) : sp.K[c]) : 0;
                if (cnt > 0)
                    tile_sum_acc<T, DEN, false, TP>(sh.u.t.tile + sp.R[c], cnt, sl, sp.S[c], tx, ty, tz, nullptr, acc);
            }
            __syncthreads();
        }
    }
    store_partials(sh, act, acc);
    __syncthreads();
    // slot o of class k4: (target group tj, component, target k of the
    // group) as in slice_sums, slices added in order from zero
    for (int o = tid; o < sp.nout[4]; o += NTT) {
        int k4 = 0;
        while (o >= sp.nout[k4 + 1]) ++k4;
        const int hc = sp.h[k4], r0 = o - sp.nout[k4];
        int k = 0;
#pragma unroll
        for (int j = 1; j < TP; ++j) k += r0 >= j * 3 * hc;
        const int rem = r0 - k * 3 * hc;
        const int comp = (rem >= hc) + (rem >= 2 * hc), tj = rem - comp * hc;
        const int j = tj + k * hc;
        if (j < STC_PICK4(a.cls.np, k4)) {
            double sum = 0.0;
            for (int q = 0; q < sp.S[k4]; ++q) sum += sh.u.red[k][comp][sp.base[k4] + q * hc + tj];
            a.alpha[(rec + (size_t)STC_PICK4(a.cls.poff, k4) + j) * 3 + comp] = sum;
        }
    }
    if (tid == 0) {
        u32 present = 0;
        for (int k = 0; k < 4; ++k)
            if (sp.tot[k]) present |= 1u << k;
        a.cls_mask[a.slot[t]] = present;
    }
    __syncthreads();
}

template <typename T, int DEN, int NT>
__global__ __launch_bounds__(NT) void k_near(EvalArgs a, u32 type_mask) {
    constexpr int TP = NEAR_TP;
    __shared__ SegShared<T, NT, TP, false> sh;
    u32 n = a.counters[C_TLIST];
    if (n > a.cap) n = a.cap;
    u32 e, e_hi;
    const int shf = a.W + 1 + a.DB;
    if (!wg_range<false>(n, a.tlist, a.tseg_end, shf, e, e_hi)) return;
    const bool rel = sizeof(T) == 4;  // FP32: coordinates relative to the target circumcentre
    while (e < e_hi) {
        const u32 t = (u32)(a.tlist[e] >> shf);
        const u32 se = (u32)a.tseg_end[t];
        const i32 tb = a.nbeg[t];
        const int nt = a.nend[t] - tb;
        const NodeGeo& gt = a.geo[t & a.node_mask];
        const double cx = rel ? gt.c[0] : 0.0, cy = rel ? gt.c[1] : 0.0, cz = rel ? gt.c[2] : 0.0;
        for (int cb = 0; cb < nt; cb += TP * NT) {
            const int ntc = (nt - cb) < TP * NT ? (nt - cb) : TP * NT;
            const TargetGroup<TP> tg(ntc, NT, cb);
            T tx[TP], ty[TP], tz[TP];
            int me[TP];
#pragma unroll
            for (int k = 0; k < TP; ++k) {
                const i32 gi = tb + tg.me[k];
                tx[k] = target_reg<T>(a.sx[gi] - cx);
                ty[k] = target_reg<T>(a.sy[gi] - cy);
                tz[k] = target_reg<T>(a.sz[gi] - cz);
                me[k] = tg.valid[k] ? tg.me[k] : -1;  // a duplicate target's exclusion never matches
            }
            double acc[TP][4];
#pragma unroll
            for (int k = 0; k < TP; ++k) acc[k][0] = acc[k][1] = acc[k][2] = acc[k][3] = 0.0;
            accumulate_entries<T, DEN>(a, a.tlist, e, se, type_mask, t, me, tg.act, tg.sl, tg.S, tx, ty, tz, cx, cy,
                                       cz, sh, acc);
            store_partials(sh, tg.act, acc);
            __syncthreads();
            // every particle's leaf has a segment (its PP entry with itself),
            // processed by one workgroup in one pass per target: this is the
            // particle's first and only write of the near-side sums
            auto add = [&](int j, int c, double v) { a.Wacc[3 * (size_t)(tb + cb + j) + c] = v; };
            slice_sums<NT, TP>(sh.u.red, tg.h, tg.S, ntc, add);
            __syncthreads();
        }
        e = se > e ? se : e + 1;  // a segment always ends after its first entry
    }
}

// One class pass of the matrix-core form over NG groups of 16 target
// points (sh.tgt): the per-lane block sums of entries [ec, ce), then (in
// FP64) the four source subgroups of a block row meet in lanes 0..15 (lane
// 4 b + j, register i: target 16 g + 4 b + i, column j) and go to the wave's
// row of sh.u.wred.  Ends with a barrier.
template <int NG, int NTT, int TP>
__device__ __forceinline__ void far_pass_mf(const EvalArgs& a, u32 ec, u32 ce, double cx, double cy, double cz,
                                            SegShared<float, NTT, TP, true>& sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, kq = lane >> 4;
    float bop[NG];
    mf32x4 acc[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        const mf32x4 tv = sh.tgt.v[16 * g + (lane & 15)];
        bop[g] = kq < 3 ? -2.f * tv[kq] : tv[3];
        acc[g] = mf32x4{0.f, 0.f, 0.f, 0.f};
    }
    accumulate_entries_mf<NG>(a, a.nlist, ec, ce, cx, cy, cz, sh, bop, acc);
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            double v = (double)acc[g][i];
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            if (lane < 16) sh.u.wred.v[w][16 * g + 4 * (lane >> 2) + i][lane & 3] = v;
        }
    __syncthreads();
}

// Target-side far field (CP and CC), one list segment per target node t:
// the node's interpolation points x~_m (its proxy points, as the upward pass
// stored them) of each degree class present receive
//   W(x~_m) = sum over the class's entries of q (y - x~_m) / den,
// written to the node's coefficient record in place of the coefficients,
// which k_far_finish forms from them.  With the learned form the classes
// present go to cls_mask[slot].
// MF: the matrix-core form (FP32 velocity, at most kMfTargets points per
// class); LEARNED: the degree classes of the learned form.
// (The matrix-core form of the plain method fits 128 VGPRs, four waves per
// SIMD; unconstrained it takes a few more and only three.)
template <typename T, int DEN, int NTT, bool MF, bool LEARNED>
__global__ __launch_bounds__(NTT) __attribute__((amdgpu_waves_per_eu((MF && !LEARNED) ? 4 : 1))) void k_far_targets(
    EvalArgs a) {
    constexpr int TP = FAR_TP;
    __shared__ SegShared<T, NTT, TP, MF> sh;
    __shared__ double wt[kMaxNp][3];
    const int tid = threadIdx.x;
    u32 n = a.counters[C_NLIST];
    if (n > a.cap) n = a.cap;
    u32 e, e_hi;
    const int shf = a.W + 1 + a.DB;  // segments by target node (all classes)
    if (!wg_range<true>(n, a.nlist, a.nseg_end, shf, e, e_hi)) return;
    const bool rel = sizeof(T) == 4;
    while (e < e_hi) {
        const u32 t = (u32)(a.nlist[e] >> shf);
        const u32 se = (u32)a.nseg_end[t];
        const NodeGeo& gt = a.geo[t & a.node_mask];
        const double cx = rel ? gt.c[0] : 0.0, cy = rel ? gt.c[1] : 0.0, cz = rel ? gt.c[2] : 0.0;
        const size_t rec = (size_t)a.slot[t] * a.NPT;
        // W(x~_m) of class c's points from entries [ec, ce), written to the
        // class's record
        auto class_values = [&](int c, u32 ec, u32 ce) {
            const int np = STC_PICK4(a.cls.np, c), poff = STC_PICK4(a.cls.poff, c);
            const Prox* __restrict__ tp = a.prox + rec + poff;
            if constexpr (MF) {
                // all points in one pass, groups of 16 (padding points at the
                // origin with |x|^2 = 1 keep every denominator positive)
                const int ng = (np + 15) >> 4;
                for (int m = tid; m < 16 * ng; m += NTT) {
                    if (m < np) {
                        const Prox pm = tp[m];
                        const float x0 = (float)(pm.x - cx), x1 = (float)(pm.y - cy), x2 = (float)(pm.z - cz);
                        const double a2 = ((double)x0 * x0 + (double)x1 * x1) + (double)x2 * x2;
                        sh.tgt.v[m] = mf32x4{x0, x1, x2, (float)a2};
                    } else {
                        sh.tgt.v[m] = mf32x4{0.f, 0.f, 0.f, 1.f};
                    }
                }
                __syncthreads();
                switch (ng) {
                    case 1: far_pass_mf<1>(a, ec, ce, cx, cy, cz, sh); break;
                    case 2: far_pass_mf<2>(a, ec, ce, cx, cy, cz, sh); break;
                    case 3: far_pass_mf<3>(a, ec, ce, cx, cy, cz, sh); break;
                    case 4: far_pass_mf<4>(a, ec, ce, cx, cy, cz, sh); break;
                    default: far_pass_mf<5>(a, ec, ce, cx, cy, cz, sh); break;
                }
                for (int o = tid; o < 3 * np; o += NTT) {
                    const int m = o / 3, cc = o - 3 * m;
                    double sc = 0.0, s3 = 0.0;
                    for (int ww = 0; ww < NTT / 64; ++ww) {
                        sc += sh.u.wred.v[ww][m][cc];
                        s3 += sh.u.wred.v[ww][m][3];
                    }
                    a.alpha[(rec + poff) * 3 + o] = sc - (double)sh.tgt.v[m][cc] * s3;
                }
                __syncthreads();
            } else {
                // target points in passes of up to TP NTT / 4 (degree 10 with
                // 256 threads: all 66 points in one pass, 33 target pairs x 7
                // slices)
                for (int cb = 0; cb < np; cb += TP * NTT / 4) {
                    const int ntc = (np - cb) < TP * NTT / 4 ? (np - cb) : TP * NTT / 4;
                    const TargetGroup<TP> tg(ntc, NTT, cb);
                    T tx[TP], ty[TP], tz[TP];
                    int nome[TP];
#pragma unroll
                    for (int k = 0; k < TP; ++k) {
                        const Prox pm = tp[tg.me[k]];
                        tx[k] = target_reg<T>(pm.x - cx);
                        ty[k] = target_reg<T>(pm.y - cy);
                        tz[k] = target_reg<T>(pm.z - cz);
                        nome[k] = -1;
                    }
                    double acc[TP][4];
#pragma unroll
                    for (int k = 0; k < TP; ++k) acc[k][0] = acc[k][1] = acc[k][2] = acc[k][3] = 0.0;
                    accumulate_entries<T, DEN>(a, a.nlist, ec, ce, 3u, 0xffffffffu, nome, tg.act, tg.sl, tg.S, tx, ty,
                                               tz, cx, cy, cz, sh, acc);
                    store_partials(sh, tg.act, acc);
                    __syncthreads();
                    auto put = [&](int j, int cc, double v) { wt[cb + j][cc] = v; };
                    slice_sums<NTT, TP>(sh.u.red, tg.h, tg.S, ntc, put);
                    __syncthreads();
                }
                for (int o = tid; o < 3 * np; o += NTT) a.alpha[(rec + poff) * 3 + o] = wt[o / 3][o % 3];
            }
        };
        if constexpr (!LEARNED) {
            class_values(0, e, se);
        } else if constexpr (!MF) {
            learned_far_values<T, DEN, NTT, TP>(a, e, se, t, rec, cx, cy, cz, sh);
        } else {
            const u32 cmask = (1u << a.DB) - 1u;
            u32 present = 0;
            u32 ec = e;
            while (ec < se) {  // the classes present, in increasing order
                const int c = (int)((a.nlist[ec] >> (a.W + 1)) & cmask);
                u32 lo = ec, hi = se;  // class(lo) == c; class(hi) > c or hi == se
                while (hi - lo > 1) {
                    const u32 mid = (lo + hi) >> 1;
                    if ((int)((a.nlist[mid] >> (a.W + 1)) & cmask) == c) lo = mid;
                    else hi = mid;
                }
                class_values(c, ec, hi);
                present |= 1u << c;
                ec = hi;
            }
            if (tid == 0) a.cls_mask[a.slot[t]] = present;
        }
        __syncthreads();
        e = se > e ? se : e + 1;  // a segment always ends after its first entry
    }
}

// i64 value of lane `src` (wave-uniform result)
__device__ __forceinline__ i64 readlane64(i64 v, int src) {
    const u32 lo = (u32)__builtin_amdgcn_readlane((int)(u32)v, src);
    const u32 hi = (u32)__builtin_amdgcn_readlane((int)(u32)((u64)v >> 32), src);
    return (i64)(((u64)hi << 32) | lo);
}

// The nodes with more than N_T particles of all levels in one index space:
// lvl_end[l] = the number of such nodes at levels <= l (each level's count
// capped at its list's capacity), filled once per workgroup (ends with a
// barrier), so that finding a node's level costs no global loads.
__device__ __forceinline__ u32 big_node_table(const EvalArgs& a, u32* lvl_end) {
    const int tid = threadIdx.x;
    if (tid <= a.L) lvl_end[tid] = a.level_big[tid] < a.per_level ? a.level_big[tid] : a.per_level;  // loads in parallel
    __syncthreads();
    if (tid == 0)
        for (int lvl = 1; lvl <= a.L; ++lvl) lvl_end[lvl] += lvl_end[lvl - 1];
    __syncthreads();
    return lvl_end[a.L];
}

// node gi of that index space
__device__ __forceinline__ i64 big_node(const EvalArgs& a, const u32* lvl_end, u32 gi) {
    int lvl = 0;
    while (gi >= lvl_end[lvl]) ++lvl;
    return a.big_list[(size_t)lvl * a.per_level + (gi - (lvl > 0 ? lvl_end[lvl - 1] : 0u))];
}

// The coefficients of every target node of the far lists from the values
// k_far_targets left in its record (Sec. 3, interpolation in triangles):
//   alpha_k = sum_m (V_ref^{-1})_km |P_m|^d W(x~_m),
// P_m = b_m1 v1 + b_m2 v2 + b_m3 v3 the unnormalised point, stored as
// c_k alpha_k (the basis multinomial folded in once per node rather than
// once per particle).  One workgroup per node with more than N_T particles
// (all levels in one index space; nodes without far-field work are
// skipped).  The product is block_matvec's (the same sums in the same
// order), with each thread's matrix entries loaded all at once before its
// FMAs when its share of the rows is at most kFinPer (degree <= 10), so that
// a node waits on one round of loads instead of a chain.
constexpr int kFinPer = 22;
__global__ __launch_bounds__(256) void k_far_finish_one_block(EvalArgs a) {
    __shared__ double w[kMaxNp][3];
    __shared__ double nd[kMaxNp];
    __shared__ double co[kMaxNp][3];
    __shared__ double red[3 * 256];
    __shared__ u32 lvl_end[kMaxLevels + 1];
    const int tid = threadIdx.x;
    const int np = a.cls.np[0], poff = a.cls.poff[0], d = a.cls.deg[0];
    const double* __restrict__ Vt = a.ref.vinvT + a.cls.qoff[0];
    int rem, k;
    const int G = div_small(256, np, rem);
    const int grp = div_small(tid, np, k);
    const int per = div_small(np + G - 1, G, rem);
    const int m0 = grp * per, m1 = (m0 + per) < np ? (m0 + per) : np;
    const bool pref = per <= kFinPer;
    const u32 total = big_node_table(a, lvl_end);
    for (u32 gi = blockIdx.x; gi < total; gi += gridDim.x) {
        const i64 node = big_node(a, lvl_end, gi);
        if (a.nseg_end[node] == 0) continue;  // no far-field work at this node
        const NodeGeo& g = a.geo[node & a.node_mask];
        const size_t rec = (size_t)a.slot[node] * a.NPT + poff;
        // this thread's matrix entries, in flight while the values arrive
        double mv[kFinPer];
        if (pref && grp < G) {
#pragma unroll
            for (int j = 0; j < kFinPer; ++j) mv[j] = (m0 + j < m1) ? Vt[(size_t)(m0 + j) * np + k] : 0.0;
        }
        for (int m = tid; m < np; m += 256) {
            double y[3];
            nd[m] = ipow(proxy_point(g, a.ref.points + 3 * (poff + m), y), d);
            w[m][0] = a.alpha[(rec + m) * 3];
            w[m][1] = a.alpha[(rec + m) * 3 + 1];
            w[m][2] = a.alpha[(rec + m) * 3 + 2];
        }
        __syncthreads();
        if (pref) {
            double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
            if (grp < G) {
#pragma unroll
                for (int j = 0; j < kFinPer; ++j) {
                    if (m0 + j < m1) {
                        const double f = mv[j] * nd[m0 + j];
                        acc0 += f * w[m0 + j][0];
                        acc1 += f * w[m0 + j][1];
                        acc2 += f * w[m0 + j][2];
                    }
                }
            }
            red[tid] = (grp < G) ? acc0 : 0.0;
            red[256 + tid] = (grp < G) ? acc1 : 0.0;
            red[512 + tid] = (grp < G) ? acc2 : 0.0;
            __syncthreads();
            if (tid < np) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    double sum = 0.0;
                    for (int gg = 0; gg < G; ++gg) sum += red[c * 256 + gg * np + tid];
                    co[tid][c] = sum;
                }
            }
            __syncthreads();
        } else {
            block_matvec<256, 3>(Vt, np, np, nd, w, red, co);
        }
        for (int q = tid; q < 3 * np; q += 256) a.alpha[rec * 3 + q] = a.ref.coef[poff + q / 3] * co[q / 3][q % 3];
        __syncthreads();
    }
}

// LDS writes of a wave visible to its other lanes: a wave's LDS operations
// execute in order, and the fences keep the compiler from moving them.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Output k of the one-class coefficient product (three components): the
// rows summed in the groups of 256 / np rows that a 256-thread workgroup's
// block_matvec forms, the groups added in order, so that the result is
// bitwise that of k_far_finish_one_block.  Vt: V^-1 transposed (np x np,
// [m][k]); nd, w: the node's scaled values.
__device__ __forceinline__ void one_class_sums(const double* Vt, int np, const double* nd, const double (*w)[3],
                                               int k, double* s) {
    int rem;
    const int G = div_small(256, np, rem);
    const int per = div_small(np + G - 1, G, rem);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll 1
    for (int gg = 0; gg < G; ++gg) {
        const int m0 = gg * per, m1 = (m0 + per) < np ? (m0 + per) : np;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll 4
        for (int m = m0; m < m1; ++m) {
            const double f = Vt[m * np + k] * nd[m];
            a0 += f * w[m][0];
            a1 += f * w[m][1];
            a2 += f * w[m][2];
        }
        s0 += a0;
        s1 += a1;
        s2 += a2;
    }
    s[0] = s0;
    s[1] = s1;
    s[2] = s2;
}

// A node's scaled values at one point: |P_m|^d and W(x~_m) (32 bytes, read
// by a wave's lanes together as two 16-byte broadcasts).
struct alignas(16) NdW {
    double nd, w[3];
};

// Every output of a node by one wave: lane l < h = ceil(np / 2) takes
// outputs l and l + h, so that each row's broadcast inputs serve two outputs
// (LDS issue, not arithmetic, bounds this product); the sums are
// one_class_sums', times c_k.
__device__ __forceinline__ void wave_one_class(const double* Vt, int np, const NdW* x, const double* coef,
                                               double* alpha_rec) {
    const int lane = threadIdx.x & 63;
    const int h = (np + 1) >> 1;
    if (lane >= h) return;
    const int k0 = lane, k1 = lane + h;
    const bool two = k1 < np;
    int rem;
    const int G = div_small(256, np, rem);
    const int per = div_small(np + G - 1, G, rem);
    double s[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
#pragma unroll 1
    for (int gg = 0; gg < G; ++gg) {
        const int m0 = gg * per, m1 = (m0 + per) < np ? (m0 + per) : np;
        double a[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
#pragma unroll 2
        for (int m = m0; m < m1; ++m) {
            const NdW xm = x[m];
            const double f0 = Vt[m * np + k0] * xm.nd;
            const double f1 = (two ? Vt[m * np + k1] : 0.0) * xm.nd;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                a[0][c] += f0 * xm.w[c];
                a[1][c] += f1 * xm.w[c];
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            s[0][c] += a[0][c];
            s[1][c] += a[1][c];
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) alpha_rec[3 * k0 + c] = coef[k0] * s[0][c];
    if (two)
#pragma unroll
        for (int c = 0; c < 3; ++c) alpha_rec[3 * k1 + c] = coef[k1] * s[1][c];
}

// The nodes with far-field work of workgroup range [c0, c0 + cnt) of the
// big-node index space, fetched by one thread each (the chain node -> its
// segment -> its slot -> its class mask is then paid once per chunk, not once
// per node): node (-1: no far work), coefficient record and classes present.
// Ends with a barrier.
constexpr int kFinChunk = 512;
struct FinNodes {
    i64 node[kFinChunk];
    u64 rec[kFinChunk];
    u32 present[kFinChunk];
};
__device__ __forceinline__ void fin_fetch_nodes(const EvalArgs& a, const u32* lvl_end, u32 c0, u32 cnt, bool learned,
                                                FinNodes& fn) {
    const int tid = threadIdx.x;
    for (u32 i = tid; i < cnt; i += blockDim.x) {
        i64 node = big_node(a, lvl_end, c0 + i);
        u64 rec = 0;
        u32 present = 0;
        if (a.nseg_end[node] == 0) {
            node = -1;  // no far-field work at this node
        } else {
            const i32 sl = a.slot[node];
            rec = (u64)sl * (u64)a.NPT;
            present = learned ? a.cls_mask[sl] : 1u;
        }
        fn.node[i] = node;
        fn.rec[i] = rec;
        fn.present[i] = present;
    }
    __syncthreads();
}

// The coefficients of every target node of the far lists (the one-class
// formula above) with V^-1 in LDS, read once per workgroup: a wave per node,
// kFinWaves nodes of a workgroup at a time, the workgroup's nodes fetched a
// chunk at a time (a workgroup per node read the 35 KB table from L2 for
// every node and waited on the node's chain of loads).  Degree <= 10 (np <= 66); larger
// degrees take k_far_finish_one_block.
constexpr int kFinWaves = 8;
constexpr int kFinNp = 66;
__global__ __launch_bounds__(64 * kFinWaves) void k_far_finish_one(EvalArgs a) {
    __shared__ double Vs[kFinNp * kFinNp];
    __shared__ NdW xv[kFinWaves][kFinNp];
    __shared__ FinNodes fn;
    __shared__ u32 lvl_end[kMaxLevels + 1];
    const int tid = threadIdx.x, lane = tid & 63, wi = tid >> 6;
    const int np = a.cls.np[0], poff = a.cls.poff[0], d = a.cls.deg[0];
    const double* __restrict__ Vt = a.ref.vinvT + a.cls.qoff[0];
#pragma unroll 9
    for (int i = tid; i < np * np; i += 64 * kFinWaves) Vs[i] = Vt[i];
    const u32 total = big_node_table(a, lvl_end);  // ends with a barrier
    // this workgroup's contiguous range of the big nodes, in chunks
    const u32 per = (total + gridDim.x - 1) / gridDim.x;
    const u32 lo = blockIdx.x * per, hi = (lo + per) < total ? (lo + per) : total;
    for (u32 c0 = lo; c0 < hi; c0 += kFinChunk) {
        const u32 cnt = (hi - c0) < (u32)kFinChunk ? (hi - c0) : (u32)kFinChunk;
        fin_fetch_nodes(a, lvl_end, c0, cnt, false, fn);
        for (u32 j = wi; j < cnt; j += kFinWaves) {
            const i64 node = fn.node[j];
            if (node < 0) continue;
            const NodeGeo& g = a.geo[node & a.node_mask];
            const size_t rec = (size_t)fn.rec[j] + poff;
            for (int m = lane; m < np; m += 64) {
                double y[3];
                NdW v;
                v.nd = ipow(proxy_point(g, a.ref.points + 3 * (poff + m), y), d);
                v.w[0] = a.alpha[(rec + m) * 3];
                v.w[1] = a.alpha[(rec + m) * 3 + 1];
                v.w[2] = a.alpha[(rec + m) * 3 + 2];
                xv[wi][m] = v;
            }
            wave_lds_sync();
            wave_one_class(Vs, np, xv[wi], a.ref.coef + poff, a.alpha + rec * 3);
            wave_lds_sync();  // the next node's values replace these
        }
        __syncthreads();  // the next chunk replaces the node list
    }
}

// the learned form's classes: degrees 4, 6, 8 and 10, 15 + 28 + 45 + 66 points
constexpr int kLearnedNpt = 154;

// The learned form folds its classes into one degree-10 record: on the
// sphere a degree-d polynomial in the barycentrics equals a degree-10 one
// (times |V b|^(10 - d) = 1, d even), so the degree-10 interpolant through
// its values at the degree-10 points reproduces it exactly (up to
// rounding); its scaled values there are
//   v_n = |P10_n|^(10 - d) sum_m T_nm |P_m|^d W(x~_m),
// T_nm = sum_k (V_ref,d^{-1})_km B_k(b_10,n) (the class's Lagrange basis at
// the degree-10 reference points; identity for degree 10), and the record is
// c_k sum_n (V_ref,10^{-1})_kn (sum over classes of v_n).  A node with
// degree-10 work only takes the one-class formula of k_far_finish_one (the
// same arithmetic, so without a network the learned context is bitwise the
// method without gating).  The tables (up_T of the lower classes, up_H)
// sit in LDS, read once per workgroup; the workgroup takes kFinBatch nodes
// at a time: a thread per (node, point) for the present classes' scaled
// values and the degree-10 points' factors, then a thread per (node,
// degree-10 point) for v (classes in order), then a thread per (node, output)
// for the product with up_H in the row groups of a 256-thread block_matvec.
constexpr int kLearnedNlow = kLearnedNpt - kFinNp;  // points of the classes below degree 10 (88)
constexpr int kFinBatch = 7;                         // nodes per round: 7 x 66 items fit 512 threads
struct LearnedFinishLds {
    double T[kLearnedNlow * kFinNp];  // up_T of classes 0..2: [poff_c + m][n]
    double H[kFinNp * kFinNp];        // up_H: [n][k]
    double xs[kFinBatch][kLearnedNpt][3];
    double sc[kFinBatch][3][kFinNp];
    double v10[kFinBatch][kFinNp][3];
};

__global__ __launch_bounds__(64 * kFinWaves) void k_far_finish_learned(EvalArgs a) {
    __shared__ LearnedFinishLds sh;
    __shared__ FinNodes fn;
    __shared__ u32 lvl_end[kMaxLevels + 1];
    const int tid = threadIdx.x;
#pragma unroll 12
    for (int i = tid; i < kLearnedNlow * kFinNp; i += 64 * kFinWaves) sh.T[i] = a.up_T[i];
#pragma unroll 9
    for (int i = tid; i < kFinNp * kFinNp; i += 64 * kFinWaves) sh.H[i] = a.up_H[i];
    const u32 total = big_node_table(a, lvl_end);  // ends with a barrier
    const int np10 = kFinNp, poff10 = kLearnedNlow, d10 = a.cls.deg[3];
    // this thread's item of the two product steps: batch node ib, point or
    // output n (ib >= kFinBatch: none).  (Two items per thread, as in
    // wave_one_class, measured slower here: 231 of the 512 threads active.)
    int n_it;
    const int ib = div_small(tid, np10, n_it);
    const u32 per = (total + gridDim.x - 1) / gridDim.x;  // this workgroup's range, in chunks
    const u32 lo = blockIdx.x * per, hi = (lo + per) < total ? (lo + per) : total;
    for (u32 c0 = lo; c0 < hi; c0 += kFinChunk) {
        const u32 cnt = (hi - c0) < (u32)kFinChunk ? (hi - c0) : (u32)kFinChunk;
        fin_fetch_nodes(a, lvl_end, c0, cnt, true, fn);
        for (u32 g0 = 0; g0 < cnt; g0 += kFinBatch) {
            // every (node, point) item of the batch's scaled values over the
            // whole workgroup
#pragma unroll 1
            for (int it = tid; it < kFinBatch * kLearnedNpt; it += 64 * kFinWaves) {
                int i;
                const int b = div_small(it, kLearnedNpt, i);
                if (g0 + b >= cnt) continue;
                const i64 node = fn.node[g0 + b];
                if (node < 0) continue;
                const u32 present = fn.present[g0 + b];
                const size_t rec = fn.rec[g0 + b];
                const NodeGeo& g = a.geo[node & a.node_mask];
                const int c = (i >= a.cls.poff[1]) + (i >= a.cls.poff[2]) + (i >= poff10);
                double (*xs)[3] = sh.xs[b];
                if (present == 8u) {  // the one-class formula: nd in sc[0], values in xs
                    if (c < 3) continue;
                    const int m = i - poff10;
                    double y[3];
                    sh.sc[b][0][m] = ipow(proxy_point(g, a.ref.points + 3 * i, y), d10);
                    xs[m][0] = a.alpha[(rec + i) * 3];
                    xs[m][1] = a.alpha[(rec + i) * 3 + 1];
                    xs[m][2] = a.alpha[(rec + i) * 3 + 2];
                    continue;
                }
                // every present class's |P_m|^d W(x~_m) at its record offsets,
                // and the degree-10 points' |P10_n|^(10 - d) of the lower classes
                const bool here = (present >> c) & 1u;
                if (!here && c < 3) continue;
                double y[3];
                const double r = proxy_point(g, a.ref.points + 3 * i, y);
                if (here) {
                    const double f = ipow(r, STC_PICK4(a.cls.deg, c));
#pragma unroll
                    for (int j = 0; j < 3; ++j) xs[i][j] = f * a.alpha[(rec + i) * 3 + j];
                }
                if (c == 3)
#pragma unroll
                    for (int k = 0; k < 3; ++k) sh.sc[b][k][i - poff10] = ipow(r, d10 - a.cls.deg[k]);
            }
            __syncthreads();
            // v10[ib][n] = the lower classes' parts in class order (the class's
            // Lagrange basis at degree-10 point n times its scaled values, times
            // the point's factor), then the degree-10 values
            if (ib < kFinBatch && g0 + ib < cnt && fn.node[g0 + ib] >= 0 && fn.present[g0 + ib] != 8u) {
                const u32 present = fn.present[g0 + ib];
                const double (*xs)[3] = sh.xs[ib];
                const int n = n_it;
                double v0 = 0.0, v1 = 0.0, v2 = 0.0;
#pragma unroll 1
                for (int k = 0; k < 3; ++k) {
                    if (!((present >> k) & 1u)) continue;
                    const int np = STC_PICK4(a.cls.np, k), poff = STC_PICK4(a.cls.poff, k);
                    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll 4
                    for (int m = 0; m < np; ++m) {
                        const double f = sh.T[(poff + m) * np10 + n];
                        a0 += f * xs[poff + m][0];
                        a1 += f * xs[poff + m][1];
                        a2 += f * xs[poff + m][2];
                    }
                    const double sk = sh.sc[ib][k][n];
                    {
#pragma clang fp contract(off)
                        v0 += a0 * sk;
                        v1 += a1 * sk;
                        v2 += a2 * sk;
                    }
                }
                if (present & 8u) {
                    v0 += xs[poff10 + n][0];
                    v1 += xs[poff10 + n][1];
                    v2 += xs[poff10 + n][2];
                }
                sh.v10[ib][n][0] = v0;
                sh.v10[ib][n][1] = v1;
                sh.v10[ib][n][2] = v2;
            }
            __syncthreads();
            // output k = n_it of node ib: c_k (V_ref,10^{-1} v)_k with up_H in
            // block_matvec's row groups, or the one-class formula
            if (ib < kFinBatch && g0 + ib < cnt && fn.node[g0 + ib] >= 0) {
                const int k = n_it;
                const size_t out = (fn.rec[g0 + ib] + poff10 + k) * 3;
                double sum[3];
                if (fn.present[g0 + ib] == 8u) {
                    one_class_sums(a.ref.vinvT + a.cls.qoff[3], np10, sh.sc[ib][0], sh.xs[ib], k, sum);
                    const double ck = a.ref.coef[poff10 + k];
                    a.alpha[out] = ck * sum[0];
                    a.alpha[out + 1] = ck * sum[1];
                    a.alpha[out + 2] = ck * sum[2];
                } else {
                    int rem;
                    const int G = div_small(256, np10, rem);
                    const int per = div_small(np10 + G - 1, G, rem);
                    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll 1
                    for (int gg = 0; gg < G; ++gg) {
                        const int m0 = gg * per, m1 = (m0 + per) < np10 ? (m0 + per) : np10;
                        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll 4
                        for (int m = m0; m < m1; ++m) {
                            const double f = sh.H[m * np10 + k];
                            a0 += f * sh.v10[ib][m][0];
                            a1 += f * sh.v10[ib][m][1];
                            a2 += f * sh.v10[ib][m][2];
                        }
                        s0 += a0;
                        s1 += a1;
                        s2 += a2;
                    }
                    a.alpha[out] = s0;
                    a.alpha[out + 1] = s1;
                    a.alpha[out + 2] = s2;
                }
            }
            __syncthreads();  // the next batch replaces these
        }
    }
}

// Interpolation to the particles and output.  For every node t holding
// particle i that received CP/CC work, W_i += sum_k B_k(b_t(x_i)) alpha_k(t)
// (the target-side interpolation of Sec. 3), per degree class; then
// u_i = -(1/4pi) x_i x W_i, scattered to input order.  A thread per particle
// in tree order; a level without nodes of more than N_T particles is skipped
// (such levels hold no target node of the proxy lists).  A wave's particles
// lie in a few consecutive nodes (mostly one at the coarse levels): the wave
// takes them one at a time, the node id read from one lane, so that the
// node's coefficients are wave-uniform: they come in through scalar loads
// and enter the FMAs as scalar operands, with only the node's lanes active.
// Per-lane copies (from LDS) would cost 64 x 8 bytes of LDS return per
// coefficient and wave, twice the FP64 work they feed.

// class of degree D (point offset poff) at one level: `has` marks a
// particle whose node nd at this level holds far-field coefficients
template <int D>
__device__ __forceinline__ void l2p_level(const EvalArgs& a, int poff, bool has, i64 nd, double x0, double x1,
                                          double x2, double& W0, double& W1, double& W2) {
    u64 rest = __ballot(has);
    while (rest != 0) {
        const i64 node = readlane64(nd, __ffsll((unsigned long long)rest) - 1);
        const bool mine = has && nd == node;
        rest &= ~__ballot(mine);
        // the node's inverse vertex matrix and coefficients: scalar loads
        const double(*__restrict__ mi)[3] = a.geo[node & a.node_mask].minv;
        const double* __restrict__ al = a.alpha + ((size_t)a.slot[node] * a.NPT + poff) * 3;
        if (mine) {
            // barycentric coordinates of the particle in the node
            const double b0 = (mi[0][0] * x0 + mi[0][1] * x1) + mi[0][2] * x2;
            const double b1 = (mi[1][0] * x0 + mi[1][1] * x1) + mi[1][2] * x2;
            const double b2 = (mi[2][0] * x0 + mi[2][1] * x1) + mi[2][2] * x2;
            double p1[D + 1], p2[D + 1];
            p1[0] = 1.0;
            p2[0] = 1.0;
#pragma unroll
            for (int t = 1; t <= D; ++t) {
                p1[t] = p1[t - 1] * b1;
                p2[t] = p2[t - 1] * b2;
            }
            // b1^i b2^j b3^(d-i-j) with a running power of b1; two
            // accumulators per component (alternating terms) shorten the
            // FMA chains
            double A0[2] = {0.0, 0.0}, A1[2] = {0.0, 0.0}, A2[2] = {0.0, 0.0};
            double pi = 1.0;
            int k = 0;
#pragma unroll
            for (int i1 = 0; i1 <= D; ++i1) {
#pragma unroll
                for (int j1 = 0; j1 <= D - i1; ++j1) {
                    const double B = pi * (p1[j1] * p2[D - i1 - j1]);
                    A0[k & 1] = __fma_rn(B, al[3 * k + 0], A0[k & 1]);
                    A1[k & 1] = __fma_rn(B, al[3 * k + 1], A1[k & 1]);
                    A2[k & 1] = __fma_rn(B, al[3 * k + 2], A2[k & 1]);
                    ++k;
                }
                pi *= b0;
            }
            W0 += A0[0] + A0[1];
            W1 += A1[0] + A1[1];
            W2 += A2[0] + A2[1];
        }
    }
}

// D: the degree of the stored far-field record (the context's degree, or 10
// for the learned form, whose classes are folded into one record)
template <int D>
__global__ __launch_bounds__(256) void k_l2p_finalize(EvalArgs a, int do_far, double* __restrict__ u, int accumulate) {
    const int tid = threadIdx.x;
    // contiguous eighths of the particles per XCD (the grid is a multiple of
    // 8): an XCD's waves then read the coefficients of its own nodes, which
    // stay in its L2 (dealt in turn, every XCD read every node's)
    const u32 blk = (gridDim.x % 8u == 0u) ? logical_block() : blockIdx.x;
    const i64 i0 = (i64)blk * blockDim.x + tid;
    const bool valid = i0 < a.n;
    const i64 i = valid ? i0 : a.n - 1;
    const double x0 = a.sx[i], x1 = a.sy[i], x2 = a.sz[i];
    double W0 = a.Wacc[3 * i], W1 = a.Wacc[3 * i + 1], W2 = a.Wacc[3 * i + 2];
    if (do_far) {
        const u32 leaf = a.leaf[i];
        const int L = a.L;
        const i64 mbase = (i64)(leaf >> a.LB) << a.NB;
        const u32 kl = leaf & ((1u << a.LB) - 1u);
        const int poff = a.cls.poff[a.ndeg - 1];
        // which of the particle's nodes hold far-field coefficients (bit =
        // level): independent loads, issued together
        u32 hb = 0u;
#pragma unroll
        for (int lvl = 0; lvl <= kMaxLevels; ++lvl) {
            const int lc = lvl < L ? lvl : L;
            const i64 nd = mbase + a.level_off_tab[lc] + (i64)(kl >> (2 * (L - lc)));
            // a level without nodes of more than N_T particles has no target
            // node of the proxy lists
            const bool lv = valid && lvl <= L && a.level_big[lc] != 0u;
            if (lv && a.nseg_end[nd] != 0) hb |= 1u << lvl;
        }
        for (int lvl = 0; lvl <= L; ++lvl) {
            if (a.level_big[lvl] == 0u) continue;  // uniform: no work at all
            const i64 nd = mbase + a.level_off_tab[lvl] + (i64)(kl >> (2 * (L - lvl)));
            l2p_level<D>(a, poff, (hb >> lvl) & 1u, nd, x0, x1, x2, W0, W1, W2);
        }
    }
    if (!valid) return;
    if (a.stream) {  // psi = W_0 / 4 pi, one value per particle
        const double p = kInv4Pi * W0;
        const i64 o = (i64)a.perm[i];
        if (accumulate) u[o] += p;
        else u[o] = p;
        return;
    }
    // u = -(1/4pi) x x W
    const double u0 = -kInv4Pi * (x1 * W2 - x2 * W1);
    const double u1 = -kInv4Pi * (x2 * W0 - x0 * W2);
    const double u2 = -kInv4Pi * (x0 * W1 - x1 * W0);
    const i64 o = 3 * (i64)a.perm[i];
    if (accumulate) {
        u[o] += u0;
        u[o + 1] += u1;
        u[o + 2] += u2;
    } else {
        u[o] = u0;
        u[o + 1] = u1;
        u[o + 2] = u2;
    }
}

// Direct sum over sources [j_lo, j_hi) for 64 TPD targets per workgroup
// (lane l holds targets l, l + 64, ...; 4 source slices per target; every
// lane of a wave reads the same staged source, an LDS broadcast, and uses it
// for its TPD targets).  Workgroup b takes target block b % tblocks and
// source chunk b / tblocks; the block index goes through the XCD-aware map
// when the grid divides by 8, so the workgroups of one XCD share a few
// source chunks in its L2.  With one chunk the velocity is written directly;
// else the chunk's W goes to part[chunk][target][3].
template <typename T, int DEN, int TPD>
__global__ __launch_bounds__(256) void k_direct(i64 n, const double* __restrict__ x, const double* __restrict__ zeta,
                                                const double* __restrict__ area, i64 m, const i64* __restrict__ targets,
                                                i64 chunk_len, u32 tblocks, double* __restrict__ u,
                                                double* __restrict__ part) {
    __shared__ Src<T> tile[256];
    __shared__ double red[TPD][3][256];
    const u32 b = (gridDim.x % 8u == 0u) ? logical_block() : blockIdx.x;
    const u32 tb = b % tblocks, ch = b / tblocks;
    const i64 j_lo = (i64)ch * chunk_len;
    const i64 j_hi = (j_lo + chunk_len) < n ? j_lo + chunk_len : n;
    const int tid = threadIdx.x;
    const int tl = tid & 63, sl = tid >> 6;
    i64 ti[TPD], gi[TPD];
    T tx[TPD], ty[TPD], tz[TPD];
    double ax[TPD], ay[TPD], az[TPD];
#pragma unroll
    for (int k = 0; k < TPD; ++k) {
        ti[k] = (i64)tb * 64 * TPD + 64 * k + tl;
        gi[k] = ti[k] < m ? (targets ? targets[ti[k]] : ti[k]) : 0;  // targets past m repeat particle 0
        tx[k] = target_reg<T>(x[3 * gi[k]]);
        ty[k] = target_reg<T>(x[3 * gi[k] + 1]);
        tz[k] = target_reg<T>(x[3 * gi[k] + 2]);
        ax[k] = ay[k] = az[k] = 0.0;
    }
    const double qscale = charge_scale<T, DEN>();
    // the next tile's source is loaded into registers before the current
    // tile is summed, so its memory latency overlaps the arithmetic
    // (the pointers stay live across the tile loop, so no register of an
    // address is reused while its load is still in flight)
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, sz = 0.0, sa = 0.0;
    const double* px = x + 3 * (j_lo + tid);
    const double* pz = zeta + (j_lo + tid);
    const double* pa = area + (j_lo + tid);
    if (j_lo + tid < j_hi) s0 = px[0], s1 = px[1], s2 = px[2], sz = pz[0], sa = pa[0];
    for (i64 j0 = j_lo; j0 < j_hi; j0 += 256) {
        if (j0 + tid < j_hi) {
            Src<T> v;
            v.x = (T)s0;
            v.y = (T)s1;
            v.z = (T)s2;
            v.q = (T)(qscale * sz * sa);
            tile[tid] = v;
        }
        __syncthreads();
        px += 3 * 256, pz += 256, pa += 256;
        if (j0 + 256 + tid < j_hi) s0 = px[0], s1 = px[1], s2 = px[2], sz = pz[0], sa = pa[0];
        const int cnt = (j_hi - j0) < 256 ? (int)(j_hi - j0) : 256;
        int sj[TPD];
        bool self_in = false;
#pragma unroll
        for (int k = 0; k < TPD; ++k) {
            const i64 d = gi[k] - j0;
            sj[k] = (d >= 0 && d < cnt) ? (int)d : -1;
            self_in |= sj[k] >= 0;
        }
        if (self_in) tile_sum<T, DEN, true, TPD>(tile, cnt, sl, 4, tx, ty, tz, sj, ax, ay, az);
        else tile_sum<T, DEN, false, TPD>(tile, cnt, sl, 4, tx, ty, tz, nullptr, ax, ay, az);
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < TPD; ++k) {
        red[k][0][tid] = ax[k];
        red[k][1][tid] = ay[k];
        red[k][2][tid] = az[k];
    }
    __syncthreads();
    if (sl == 0) {
#pragma unroll
        for (int k = 0; k < TPD; ++k) {
            if (ti[k] >= m) continue;
            double W0 = 0.0, W1 = 0.0, W2 = 0.0;
            for (int q = 0; q < 4; ++q) {
                W0 += red[k][0][q * 64 + tl];
                W1 += red[k][1][q * 64 + tl];
                W2 += red[k][2][q * 64 + tl];
            }
            if (part) {
                double* p = part + 3 * ((i64)ch * m + ti[k]);
                p[0] = W0;
                p[1] = W1;
                p[2] = W2;
            } else if constexpr (DEN >= DEN_LOG_DOT) {
                u[ti[k]] = kInv4Pi * W0;
            } else {
                const double xg0 = x[3 * gi[k]], xg1 = x[3 * gi[k] + 1], xg2 = x[3 * gi[k] + 2];
                u[3 * ti[k] + 0] = -kInv4Pi * (xg1 * W2 - xg2 * W1);
                u[3 * ti[k] + 1] = -kInv4Pi * (xg2 * W0 - xg0 * W2);
                u[3 * ti[k] + 2] = -kInv4Pi * (xg0 * W1 - xg1 * W0);
            }
        }
    }
}

// sum of the chunks' W in chunk order (deterministic), then the cross product
__global__ __launch_bounds__(256) void k_direct_reduce(const double* __restrict__ x, i64 m,
                                                       const i64* __restrict__ targets, u32 chunks,
                                                       const double* __restrict__ part, int stream,
                                                       double* __restrict__ u) {
    const i64 ti = (i64)blockIdx.x * 256 + threadIdx.x;
    if (ti >= m) return;
    const i64 gi = targets ? targets[ti] : ti;
    double W0 = 0.0, W1 = 0.0, W2 = 0.0;
    for (u32 c = 0; c < chunks; ++c) {
        const double* p = part + 3 * ((i64)c * m + ti);
        W0 += p[0];
        W1 += p[1];
        W2 += p[2];
    }
    if (stream) {
        u[ti] = kInv4Pi * W0;
        return;
    }
    const double xg0 = x[3 * gi], xg1 = x[3 * gi + 1], xg2 = x[3 * gi + 2];
    u[3 * ti + 0] = -kInv4Pi * (xg1 * W2 - xg2 * W1);
    u[3 * ti + 1] = -kInv4Pi * (xg2 * W0 - xg0 * W2);
    u[3 * ti + 2] = -kInv4Pi * (xg0 * W1 - xg1 * W0);
}

}  // namespace

namespace {
template <int NTT>
void near_shape(hipStream_t s, const EvalArgs& a, u32 type_mask) {
    const dim3 g(a.near_grid), b(NTT);
    if (a.stream) {
        if (a.precision == STC_FP32) hipLaunchKernelGGL((k_near<float, DEN_LOG_DIST2, NTT>), g, b, 0, s, a, type_mask);
        else if (a.denominator == STC_DEN_DIST2)
            hipLaunchKernelGGL((k_near<double, DEN_LOG_DIST2, NTT>), g, b, 0, s, a, type_mask);
        else hipLaunchKernelGGL((k_near<double, DEN_LOG_DOT, NTT>), g, b, 0, s, a, type_mask);
        return;
    }
    if (a.precision == STC_FP32) hipLaunchKernelGGL((k_near<float, STC_DEN_DIST2, NTT>), g, b, 0, s, a, type_mask);
    else if (a.denominator == STC_DEN_DIST2)
        hipLaunchKernelGGL((k_near<double, STC_DEN_DIST2, NTT>), g, b, 0, s, a, type_mask);
    else hipLaunchKernelGGL((k_near<double, STC_DEN_DOT, NTT>), g, b, 0, s, a, type_mask);
}

template <int NTT>
void far_shape(hipStream_t s, const EvalArgs& a) {
    const dim3 g(a.far_grid), b(NTT);
    if (a.stream) {  // (never with the learned form)
        if (a.precision == STC_FP32)
            hipLaunchKernelGGL((k_far_targets<float, DEN_LOG_DIST2, NTT, false, false>), g, b, 0, s, a);
        else if (a.denominator == STC_DEN_DIST2)
            hipLaunchKernelGGL((k_far_targets<double, DEN_LOG_DIST2, NTT, false, false>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_far_targets<double, DEN_LOG_DOT, NTT, false, false>), g, b, 0, s, a);
        return;
    }
    const bool learned = a.DB != 0;
    if (a.precision == STC_FP32) {
        // the matrix-core form covers classes of up to kMfTargets points
        constexpr bool MF = STC_FAR_MFMA != 0;
        if (MF && a.cls.np[a.ndeg - 1] <= kMfTargets) {
            if (learned) hipLaunchKernelGGL((k_far_targets<float, STC_DEN_DIST2, NTT, MF, true>), g, b, 0, s, a);
            else hipLaunchKernelGGL((k_far_targets<float, STC_DEN_DIST2, NTT, MF, false>), g, b, 0, s, a);
        } else {
            if (learned) hipLaunchKernelGGL((k_far_targets<float, STC_DEN_DIST2, NTT, false, true>), g, b, 0, s, a);
            else hipLaunchKernelGGL((k_far_targets<float, STC_DEN_DIST2, NTT, false, false>), g, b, 0, s, a);
        }
    } else if (a.denominator == STC_DEN_DIST2) {
        if (learned) hipLaunchKernelGGL((k_far_targets<double, STC_DEN_DIST2, NTT, false, true>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_far_targets<double, STC_DEN_DIST2, NTT, false, false>), g, b, 0, s, a);
    } else {
        if (learned) hipLaunchKernelGGL((k_far_targets<double, STC_DEN_DOT, NTT, false, true>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_far_targets<double, STC_DEN_DOT, NTT, false, false>), g, b, 0, s, a);
    }
}
}  // namespace

// workgroup sizes 128, 256 and 512 are built; the caller validates the shape
void launch_near(hipStream_t s, const EvalArgs& a, u32 type_mask) {
    if (a.near_threads == 512) near_shape<512>(s, a, type_mask);
    else if (a.near_threads == 128) near_shape<128>(s, a, type_mask);
    else near_shape<256>(s, a, type_mask);
}

void launch_far_targets(hipStream_t s, const EvalArgs& a) {
    if (a.far_threads == 512) far_shape<512>(s, a);
    else if (a.far_threads == 128) far_shape<128>(s, a);
    else far_shape<256>(s, a);
}

void launch_far_finish(hipStream_t s, const EvalArgs& a) {
    const u32 cus = (u32)std::max(a.cus, 1);
    if (a.DB != 0) {  // 140 KB of LDS: one workgroup per CU
        hipLaunchKernelGGL(k_far_finish_learned, dim3(cus), dim3(64 * kFinWaves), 0, s, a);
        return;
    }
    if (a.cls.np[0] <= kFinNp) {  // 62 KB of LDS: two workgroups per CU
        hipLaunchKernelGGL(k_far_finish_one, dim3(2 * cus), dim3(64 * kFinWaves), 0, s, a);
        return;
    }
    const unsigned grid = (unsigned)std::min<u32>(std::max<u32>(a.per_level, 1u), 2048u);
    hipLaunchKernelGGL(k_far_finish_one_block, dim3(grid), dim3(256), 0, s, a);
}

void launch_l2p_finalize(hipStream_t s, const EvalArgs& a, bool do_far, double* d_u, bool accumulate) {
    if (a.n <= 0) return;
    const dim3 g((unsigned)(((a.n + 255) / 256 + 7) / 8 * 8)), b(256);
    const int f = do_far ? 1 : 0, acc = accumulate ? 1 : 0;
    switch (a.cls.deg[a.ndeg - 1]) {
#define STC_L2P_CASE(D) \
    case D: hipLaunchKernelGGL((k_l2p_finalize<D>), g, b, 0, s, a, f, d_u, acc); break;
        STC_L2P_CASE(1) STC_L2P_CASE(2) STC_L2P_CASE(3) STC_L2P_CASE(4) STC_L2P_CASE(5) STC_L2P_CASE(6)
        STC_L2P_CASE(7) STC_L2P_CASE(8) STC_L2P_CASE(9) STC_L2P_CASE(10) STC_L2P_CASE(11) STC_L2P_CASE(12)
        STC_L2P_CASE(13) STC_L2P_CASE(14)
#undef STC_L2P_CASE
        default: break;
    }
}

// targets per lane of the direct-sum kernel (two per lane halve the LDS
// reads but cost a wave per SIMD; measured 5-10% slower in both precisions)
constexpr int DIRECT_TP32 = 1;
constexpr int DIRECT_TP64 = 1;

int direct_targets_per_block(int precision) {
    return 64 * (precision == STC_FP32 ? DIRECT_TP32 : DIRECT_TP64);
}

// Workgroups of the direct-sum kernel that fit on one CU at once.
int direct_blocks_per_cu(int precision, int denominator) {
    int nb = 0;
    hipError_t e;
    if (precision == STC_FP32)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_direct<float, STC_DEN_DIST2, DIRECT_TP32>, 256, 0);
    else if (denominator == STC_DEN_DIST2)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_direct<double, STC_DEN_DIST2, DIRECT_TP64>, 256, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_direct<double, STC_DEN_DOT, DIRECT_TP64>, 256, 0);
    if (e != hipSuccess || nb < 1) {
        (void)hipGetLastError();
        return 1;
    }
    return nb;
}

// Number of source chunks for m targets and n sources: about four times as
// many workgroups as fit on the chip at once (cus x blocks_per_cu), each
// chunk at least 2048 sources.  Workgroups of one round share the SIMDs
// unevenly and finish at different times; with several rounds the free
// slots take new workgroups, so the chip stays full to the end (measured on
// 4096 targets: 1.02 ms in one round, 0.87 ms in four).
void direct_split(i64 n, i64 m, int cus, int blocks_per_cu, int targets_per_block, u32* chunks, i64* chunk_len) {
    const i64 tblocks = (m + targets_per_block - 1) / targets_per_block;
    const i64 want = 4 * (i64)(cus > 0 ? cus : 1) * (blocks_per_cu > 0 ? blocks_per_cu : 1);
    i64 c = want / tblocks;
    const i64 cmax = (n + 2047) / 2048;
    if (c > cmax) c = cmax;
    if (c < 1) c = 1;
    i64 len = (n + c - 1) / c;
    len = (len + 255) / 256 * 256;
    c = (n + len - 1) / len;
    *chunks = (u32)c;
    *chunk_len = len;
}

void launch_direct(hipStream_t s, i64 n, const double* x, const double* zeta, const double* area, i64 m,
                   const i64* targets, int precision, int denominator, u32 chunks, i64 chunk_len, double* part,
                   double* u, int stream) {
    if (m <= 0) return;
    const int tpb = direct_targets_per_block(precision);
    const u32 tblocks = (u32)((m + tpb - 1) / tpb);
    if (!part) chunks = 1, chunk_len = n;
    double* pp = chunks > 1 ? part : nullptr;
    const dim3 g(tblocks * chunks), b(256);
    if (stream && precision == STC_FP32)
        hipLaunchKernelGGL((k_direct<float, DEN_LOG_DIST2, DIRECT_TP32>), g, b, 0, s, n, x, zeta, area, m, targets,
                           chunk_len, tblocks, u, pp);
    else if (stream && denominator == STC_DEN_DIST2)
        hipLaunchKernelGGL((k_direct<double, DEN_LOG_DIST2, DIRECT_TP64>), g, b, 0, s, n, x, zeta, area, m, targets,
                           chunk_len, tblocks, u, pp);
    else if (stream)
        hipLaunchKernelGGL((k_direct<double, DEN_LOG_DOT, DIRECT_TP64>), g, b, 0, s, n, x, zeta, area, m, targets,
                           chunk_len, tblocks, u, pp);
    else if (precision == STC_FP32)
        hipLaunchKernelGGL((k_direct<float, STC_DEN_DIST2, DIRECT_TP32>), g, b, 0, s, n, x, zeta, area, m, targets, chunk_len,
                           tblocks, u, pp);
    else if (denominator == STC_DEN_DIST2)
        hipLaunchKernelGGL((k_direct<double, STC_DEN_DIST2, DIRECT_TP64>), g, b, 0, s, n, x, zeta, area, m, targets, chunk_len,
                           tblocks, u, pp);
    else
        hipLaunchKernelGGL((k_direct<double, STC_DEN_DOT, DIRECT_TP64>), g, b, 0, s, n, x, zeta, area, m, targets, chunk_len,
                           tblocks, u, pp);
    if (pp)
        hipLaunchKernelGGL(k_direct_reduce, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, x, m, targets, chunks,
                           pp, stream, u);
}

}  // namespace stc
