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
// Segment kernels run one wave per workgroup.  A persistent grid splits the
// target-sorted list into equal contiguous ranges of entries; a workgroup
// handles every target whose run of entries starts inside its range.  The
// block -> range map is XCD aware (consecutive ranges, i.e. neighbouring
// triangles that share sources, run on the same XCD and its L2).  Sources
// are staged into 256-entry LDS tiles; lanes split as (target, source slice).
// FP32 mode: coordinates relative to the target triangle's circumcentre,
// rounded from FP64; partial sums per tile in FP32, added into FP64.
#include "common.hpp"
#include "kernels.hpp"
#include "stc.h"

namespace stc {

namespace {

constexpr int TILE = 256;

template <typename T>
struct Src {
    T x, y, z, q;
};

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

// sum over staged sources j = sl, sl + S, ... < cnt
template <typename T, int DEN, bool SELF>
__device__ __forceinline__ void tile_sum(const Src<T>* __restrict__ tile, int cnt, int sl, int S, T tx, T ty, T tz,
                                         int self_j, double& ax, double& ay, double& az) {
    T px = T(0), py = T(0), pz = T(0);
    for (int j = sl; j < cnt; j += S) {
        const Src<T> s = tile[j];
        const T dx = s.x - tx, dy = s.y - ty, dz = s.z - tz;
        T den;
        if (DEN == STC_DEN_DIST2) den = dx * dx + dy * dy + dz * dz;  // charges carry the factor 2
        else den = T(1) - (tx * s.x + ty * s.y + tz * s.z);
        T q = s.q;
        if (SELF && j == self_j) {  // the j = i term is excluded
            den = T(1);
            q = T(0);
        }
        const T w = q * rcp_t<T>(den);
        px += w * dx;
        py += w * dy;
        pz += w * dz;
    }
    ax += (double)px;
    ay += (double)py;
    az += (double)pz;
}

__device__ __forceinline__ u32 logical_block() {
    const u32 G = gridDim.x, b = blockIdx.x;
    return (b % 8u) * (G / 8u) + (b / 8u);
}

// stage source l of an entry into tile slot `slot`
template <typename T>
__device__ __forceinline__ void stage(const EvalArgs& a, int type, u32 s, i32 first, int l, double cx, double cy,
                                      double cz, double qscale, Src<T>* tile, int slot) {
    Src<T> v;
    if (type == 0) {
        const i32 j = first + l;
        v.x = (T)(a.sx[j] - cx);
        v.y = (T)(a.sy[j] - cy);
        v.z = (T)(a.sz[j] - cz);
        v.q = (T)(qscale * a.sq[j]);
    } else {
        double y[3];
        proxy_point(a.geo[s], a.ref.points + 3 * l, y);
        v.x = (T)(y[0] - cx);
        v.y = (T)(y[1] - cy);
        v.z = (T)(y[2] - cz);
        v.q = (T)(qscale * a.wq[(size_t)s * a.ref.np + l]);
    }
    tile[slot] = v;
}

// Accumulates, for the targets (tx, ty, tz) of this lane, every entry of
// [e0, e1) in `list` whose type bit is in type_mask.  self_t: target node id
// for PP self exclusion (0xffffffff: none), me: the lane's target index in
// that node.
template <typename T, int DEN>
__device__ void accumulate_entries(const EvalArgs& a, const u64* __restrict__ list, u32 e0, u32 e1, u32 type_mask,
                                   u32 self_t, int me, bool act, int sl, int S, T tx, T ty, T tz, double cx,
                                   double cy, double cz, Src<T>* tile, double& ax, double& ay, double& az) {
    const int lane = threadIdx.x;
    const u64 mask = ((u64)1 << a.W) - 1;
    const double qscale = (DEN == STC_DEN_DIST2) ? 2.0 : 1.0;
    int fill = 0;
    for (u32 e = e0; e < e1; ++e) {
        const u64 key = list[e];
        const int type = (int)((key >> a.W) & 1u);
        const u32 s = (u32)(key & mask);
        if (!((type_mask >> type) & 1u)) continue;
        const int nsrc = type == 0 ? (a.nend[s] - a.nbeg[s]) : a.ref.np;
        const i32 first = type == 0 ? a.nbeg[s] : 0;
        if (type == 0 && s == self_t) {
            if (fill > 0) {
                __syncthreads();
                if (act) tile_sum<T, DEN, false>(tile, fill, sl, S, tx, ty, tz, -1, ax, ay, az);
                __syncthreads();
                fill = 0;
            }
            for (int j0 = 0; j0 < nsrc; j0 += TILE) {
                const int cnt = (nsrc - j0) < TILE ? (nsrc - j0) : TILE;
                for (int l = lane; l < cnt; l += 64) stage<T>(a, 0, s, first, j0 + l, cx, cy, cz, qscale, tile, l);
                __syncthreads();
                if (act) tile_sum<T, DEN, true>(tile, cnt, sl, S, tx, ty, tz, me - j0, ax, ay, az);
                __syncthreads();
            }
            continue;
        }
        int off = 0;
        while (off < nsrc) {
            const int room = TILE - fill;
            const int take = (nsrc - off) < room ? (nsrc - off) : room;
            for (int l = lane; l < take; l += 64) stage<T>(a, type, s, first, off + l, cx, cy, cz, qscale, tile, fill + l);
            fill += take;
            off += take;
            if (fill == TILE) {
                __syncthreads();
                if (act) tile_sum<T, DEN, false>(tile, fill, sl, S, tx, ty, tz, -1, ax, ay, az);
                __syncthreads();
                fill = 0;
            }
        }
    }
    if (fill > 0) {
        __syncthreads();
        if (act) tile_sum<T, DEN, false>(tile, fill, sl, S, tx, ty, tz, -1, ax, ay, az);
        __syncthreads();
    }
}

template <typename T, int DEN>
__global__ __launch_bounds__(64) void k_near(EvalArgs a, u32 type_mask) {
    __shared__ Src<T> tile[TILE];
    __shared__ double red[3][64];
    const int lane = threadIdx.x;
    u32 n = a.counters[C_TLIST];
    if (n > a.cap) n = a.cap;
    const u32 G = gridDim.x;
    const u32 chunk = (n + G - 1) / G;
    const u64 lo = (u64)logical_block() * chunk;
    if (lo >= n) return;
    u32 e = (u32)lo;
    const u32 e_hi = (u64)e + chunk < n ? e + chunk : n;
    const int sh = a.W + 1;
    if (e > 0 && (a.tlist[e] >> sh) == (a.tlist[e - 1] >> sh)) e = (u32)a.tseg_end[a.tlist[e] >> sh];
    const bool rel = sizeof(T) == 4;  // FP32: coordinates relative to the target circumcentre
    while (e < e_hi) {
        const u32 t = (u32)(a.tlist[e] >> sh);
        const u32 se = (u32)a.tseg_end[t];
        const i32 tb = a.nbeg[t];
        const int nt = a.nend[t] - tb;
        const double cx = rel ? a.geo[t].c[0] : 0.0, cy = rel ? a.geo[t].c[1] : 0.0, cz = rel ? a.geo[t].c[2] : 0.0;
        for (int cb = 0; cb < nt; cb += 64) {
            const int ntc = (nt - cb) < 64 ? (nt - cb) : 64;
            const int S = 64 / ntc;
            const int ti = lane % ntc, sl = lane / ntc;
            const bool act = sl < S;
            const int me = cb + ti;
            const i32 gi = tb + me;
            const T tx = (T)(a.sx[gi] - cx), ty = (T)(a.sy[gi] - cy), tz = (T)(a.sz[gi] - cz);
            double ax = 0.0, ay = 0.0, az = 0.0;
            accumulate_entries<T, DEN>(a, a.tlist, e, se, type_mask, t, me, act, sl, S, tx, ty, tz, cx, cy, cz, tile,
                                       ax, ay, az);
            red[0][lane] = act ? ax : 0.0;
            red[1][lane] = act ? ay : 0.0;
            red[2][lane] = act ? az : 0.0;
            __syncthreads();
            if (act && sl == 0) {
                double sx = 0.0, sy = 0.0, sz = 0.0;
                for (int k = 0; k < S; ++k) {
                    sx += red[0][k * ntc + ti];
                    sy += red[1][k * ntc + ti];
                    sz += red[2][k * ntc + ti];
                }
                a.Wacc[3 * (size_t)gi + 0] += sx;
                a.Wacc[3 * (size_t)gi + 1] += sy;
                a.Wacc[3 * (size_t)gi + 2] += sz;
            }
            __syncthreads();
        }
        e = se > e ? se : e + 1;  // a segment always ends after its first entry
    }
}

template <typename T, int DEN>
__global__ __launch_bounds__(64) void k_far_targets(EvalArgs a) {
    __shared__ Src<T> tile[TILE];
    __shared__ double red[3][64];
    __shared__ double wt[kMaxNp][3];
    __shared__ double nd[kMaxNp];
    const int lane = threadIdx.x;
    u32 n = a.counters[C_NLIST];
    if (n > a.cap) n = a.cap;
    const u32 G = gridDim.x;
    const u32 chunk = (n + G - 1) / G;
    const u64 lo = (u64)logical_block() * chunk;
    if (lo >= n) return;
    u32 e = (u32)lo;
    const u32 e_hi = (u64)e + chunk < n ? e + chunk : n;
    const int sh = a.W + 1;
    if (e > 0 && (a.nlist[e] >> sh) == (a.nlist[e - 1] >> sh)) e = (u32)a.nseg_end[a.nlist[e] >> sh];
    const bool rel = sizeof(T) == 4;
    const int np = a.ref.np, d = a.ref.degree;
    while (e < e_hi) {
        const u32 t = (u32)(a.nlist[e] >> sh);
        const u32 se = (u32)a.nseg_end[t];
        const NodeGeo& gt = a.geo[t];
        const double cx = rel ? gt.c[0] : 0.0, cy = rel ? gt.c[1] : 0.0, cz = rel ? gt.c[2] : 0.0;
        for (int cb = 0; cb < np; cb += 64) {
            const int ntc = (np - cb) < 64 ? (np - cb) : 64;
            const int S = 64 / ntc;
            const int ti = lane % ntc, sl = lane / ntc;
            const bool act = sl < S;
            const int me = cb + ti;
            double y[3];
            const double nrm = proxy_point(gt, a.ref.points + 3 * me, y);
            if (act && sl == 0) nd[me] = ipow(nrm, d);
            const T tx = (T)(y[0] - cx), ty = (T)(y[1] - cy), tz = (T)(y[2] - cz);
            double ax = 0.0, ay = 0.0, az = 0.0;
            accumulate_entries<T, DEN>(a, a.nlist, e, se, 3u, 0xffffffffu, me, act, sl, S, tx, ty, tz, cx, cy, cz,
                                       tile, ax, ay, az);
            red[0][lane] = act ? ax : 0.0;
            red[1][lane] = act ? ay : 0.0;
            red[2][lane] = act ? az : 0.0;
            __syncthreads();
            if (act && sl == 0) {
                double sx = 0.0, sy = 0.0, sz = 0.0;
                for (int k = 0; k < S; ++k) {
                    sx += red[0][k * ntc + ti];
                    sy += red[1][k * ntc + ti];
                    sz += red[2][k * ntc + ti];
                }
                wt[me][0] = sx;
                wt[me][1] = sy;
                wt[me][2] = sz;
            }
            __syncthreads();
        }
        // alpha_k = sum_n (V_ref^{-1})_{kn} |b_n1 v1 + b_n2 v2 + b_n3 v3|^d W(x~_n)
        for (int k = lane; k < np; k += 64) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
            const double* vr = a.ref.vinv + (size_t)k * np;
            for (int m = 0; m < np; ++m) {
                const double c = vr[m] * nd[m];
                s0 += c * wt[m][0];
                s1 += c * wt[m][1];
                s2 += c * wt[m][2];
            }
            double* out = a.alpha + ((size_t)t * np + k) * 3;
            out[0] = s0;
            out[1] = s1;
            out[2] = s2;
        }
        __syncthreads();
        e = se > e ? se : e + 1;  // a segment always ends after its first entry
    }
}

template <int D>
__global__ __launch_bounds__(256) void k_l2p_finalize(EvalArgs a, int do_far, double* __restrict__ u, int accumulate) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const double x0 = a.sx[i], x1 = a.sy[i], x2 = a.sz[i];
    double W0 = a.Wacc[3 * i], W1 = a.Wacc[3 * i + 1], W2 = a.Wacc[3 * i + 2];
    if (do_far) {
        const u32 leaf = a.leaf[i];
        const int L = a.L;
        constexpr int NP = (D + 1) * (D + 2) / 2;
        for (int lvl = 0; lvl <= L; ++lvl) {
            const i64 node = a.level_off_tab[lvl] + (i64)(leaf >> (2 * (L - lvl)));
            if (a.nseg_end[node] == 0) continue;
            const NodeGeo& g = a.geo[node];
            double P[3][D + 1];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double be = (g.minv[c][0] * x0 + g.minv[c][1] * x1) + g.minv[c][2] * x2;
                P[c][0] = 1.0;
#pragma unroll
                for (int t = 1; t <= D; ++t) P[c][t] = P[c][t - 1] * be;
            }
            const double* al = a.alpha + (size_t)node * NP * 3;
            int k = 0;
#pragma unroll
            for (int i1 = 0; i1 <= D; ++i1) {
#pragma unroll
                for (int j1 = 0; j1 <= D - i1; ++j1) {
                    const double B = a.ref.coef[k] * (P[0][i1] * P[1][j1] * P[2][D - i1 - j1]);
                    W0 += B * al[3 * k];
                    W1 += B * al[3 * k + 1];
                    W2 += B * al[3 * k + 2];
                    ++k;
                }
            }
        }
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

// Direct sum: 64 targets x 4 source slices per workgroup, 256-source LDS tiles.
template <typename T, int DEN>
__global__ __launch_bounds__(256) void k_direct(i64 n, const double* __restrict__ x, const double* __restrict__ zeta,
                                                const double* __restrict__ area, i64 m, const i64* __restrict__ targets,
                                                double* __restrict__ u) {
    __shared__ Src<T> tile[256];
    __shared__ double red[3][256];
    const int tid = threadIdx.x;
    const int tl = tid & 63, sl = tid >> 6;
    const i64 ti = (i64)blockIdx.x * 64 + tl;
    const bool act = ti < m;
    const i64 gi = act ? (targets ? targets[ti] : ti) : 0;
    const double xg0 = x[3 * gi], xg1 = x[3 * gi + 1], xg2 = x[3 * gi + 2];
    const T tx = (T)xg0, ty = (T)xg1, tz = (T)xg2;
    const double qscale = (DEN == STC_DEN_DIST2) ? 2.0 : 1.0;
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (i64 j0 = 0; j0 < n; j0 += 256) {
        const i64 j = j0 + tid;
        if (j < n) {
            Src<T> v;
            v.x = (T)x[3 * j];
            v.y = (T)x[3 * j + 1];
            v.z = (T)x[3 * j + 2];
            v.q = (T)(qscale * zeta[j] * area[j]);
            tile[tid] = v;
        }
        __syncthreads();
        const int cnt = (n - j0) < 256 ? (int)(n - j0) : 256;
        const i64 self = gi - j0;
        if (act) {
            if (self >= 0 && self < cnt) tile_sum<T, DEN, true>(tile, cnt, sl, 4, tx, ty, tz, (int)self, ax, ay, az);
            else tile_sum<T, DEN, false>(tile, cnt, sl, 4, tx, ty, tz, -1, ax, ay, az);
        }
        __syncthreads();
    }
    red[0][tid] = ax;
    red[1][tid] = ay;
    red[2][tid] = az;
    __syncthreads();
    if (act && sl == 0) {
        double W0 = 0.0, W1 = 0.0, W2 = 0.0;
        for (int k = 0; k < 4; ++k) {
            W0 += red[0][k * 64 + tl];
            W1 += red[1][k * 64 + tl];
            W2 += red[2][k * 64 + tl];
        }
        u[3 * ti + 0] = -kInv4Pi * (xg1 * W2 - xg2 * W1);
        u[3 * ti + 1] = -kInv4Pi * (xg2 * W0 - xg0 * W2);
        u[3 * ti + 2] = -kInv4Pi * (xg0 * W1 - xg1 * W0);
    }
}

}  // namespace

void launch_near(hipStream_t s, const EvalArgs& a, u32 type_mask) {
    const dim3 g(a.grid), b(64);
    if (a.precision == STC_FP32) hipLaunchKernelGGL((k_near<float, STC_DEN_DIST2>), g, b, 0, s, a, type_mask);
    else if (a.denominator == STC_DEN_DIST2) hipLaunchKernelGGL((k_near<double, STC_DEN_DIST2>), g, b, 0, s, a, type_mask);
    else hipLaunchKernelGGL((k_near<double, STC_DEN_DOT>), g, b, 0, s, a, type_mask);
}

void launch_far_targets(hipStream_t s, const EvalArgs& a) {
    const dim3 g(a.grid), b(64);
    if (a.precision == STC_FP32) hipLaunchKernelGGL((k_far_targets<float, STC_DEN_DIST2>), g, b, 0, s, a);
    else if (a.denominator == STC_DEN_DIST2) hipLaunchKernelGGL((k_far_targets<double, STC_DEN_DIST2>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_far_targets<double, STC_DEN_DOT>), g, b, 0, s, a);
}

void launch_l2p_finalize(hipStream_t s, const EvalArgs& a, bool do_far, double* d_u, bool accumulate) {
    if (a.n <= 0) return;
    const dim3 g((unsigned)((a.n + 255) / 256)), b(256);
    const int f = do_far ? 1 : 0, acc = accumulate ? 1 : 0;
    switch (a.ref.degree) {
#define STC_L2P_CASE(D) \
    case D: hipLaunchKernelGGL((k_l2p_finalize<D>), g, b, 0, s, a, f, d_u, acc); break;
        STC_L2P_CASE(1) STC_L2P_CASE(2) STC_L2P_CASE(3) STC_L2P_CASE(4) STC_L2P_CASE(5) STC_L2P_CASE(6)
        STC_L2P_CASE(7) STC_L2P_CASE(8) STC_L2P_CASE(9) STC_L2P_CASE(10) STC_L2P_CASE(11) STC_L2P_CASE(12)
        STC_L2P_CASE(13) STC_L2P_CASE(14)
#undef STC_L2P_CASE
        default: break;
    }
}

void launch_direct(hipStream_t s, i64 n, const double* x, const double* zeta, const double* area, i64 m,
                   const i64* targets, int precision, int denominator, double* u) {
    if (m <= 0) return;
    const dim3 g((unsigned)((m + 63) / 64)), b(256);
    if (precision == STC_FP32) hipLaunchKernelGGL((k_direct<float, STC_DEN_DIST2>), g, b, 0, s, n, x, zeta, area, m, targets, u);
    else if (denominator == STC_DEN_DIST2) hipLaunchKernelGGL((k_direct<double, STC_DEN_DIST2>), g, b, 0, s, n, x, zeta, area, m, targets, u);
    else hipLaunchKernelGGL((k_direct<double, STC_DEN_DOT>), g, b, 0, s, n, x, zeta, area, m, targets, u);
}

}  // namespace stc
