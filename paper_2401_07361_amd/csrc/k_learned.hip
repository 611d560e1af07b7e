// Gated traversal of the learned form.  A first traversal with the wider
// acceptance parameter theta_max collects candidate pairs: node pairs that
// are well separated and have a side with more than N_T particles (the
// pairs the method would approximate).  For each candidate a small network
// (k_mlp.hip) reads 12 cluster summaries and predicts whether to accept the
// approximation and at which interpolation degree (4, 6, 8 or 10).
// Accepted pairs enter the lists with that degree class; rejected pairs are
// handed to the plain traversal (theta, the fallback degree), which refines
// them exactly as the fixed-degree method would.
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "kernels.hpp"

namespace stc {

namespace {

// Per node: sum of |q| and of q over its particles, level by level from the
// depth limit up (a node sums its children's sums, or its particles when it
// holds few or is at the depth limit), so the order of additions is fixed.
__global__ __launch_bounds__(256) void k_qsum_level(i64 node0, i64 nn, int lvl, int L, i64 child_off,
                                                     const i32* __restrict__ nbeg, const i32* __restrict__ nend,
                                                     const double* __restrict__ q, double* __restrict__ qabs,
                                                     double* __restrict__ qsum) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nn) return;
    const i64 nd = node0 + i;
    const i32 b = nbeg[nd], e = nend[nd];
    double sa = 0.0, ss = 0.0;
    if (e > b) {
        if (lvl == L || e - b <= 64) {
            for (i32 j = b; j < e; ++j) {
                sa += fabs(q[j]);
                ss += q[j];
            }
        } else {
            for (int c = 0; c < 4; ++c) {
                const i64 cid = child_off + 4 * i + c;
                sa += qabs[cid];
                ss += qsum[cid];
            }
        }
    }
    qabs[nd] = sa;
    qsum[nd] = ss;
}

__device__ __forceinline__ u16 f2bf(float f) {
    u32 u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}

__device__ __forceinline__ float lg10(double v) { return (float)log10(v > 1e-30 ? v : 1e-30); }

// The 12 features of candidate (t, s), rounded to BF16:
//   0 [n_t > N_T]           1 [n_s > N_T]          2 level_t / 8     3 level_s / 8
//   4 r_t / R               5 r_s / R              6 (r_t + r_s) / R (the MAC ratio)
//   7 -log10 R / 2          8 log10(Q_s / Q) / 8 + 1                 9 |sum_s q| / Q_s
//  10 log10(|w^(4)|_1 / Q_s) / 2 (0 for a small source)             11 log10(Q_t / Q) / 8 + 1
// with Q_x = sum of |q| over node x, Q over all particles, w^(4) the
// source's degree-4 proxy charges, R the chord between the circumcentres.
__global__ __launch_bounds__(256) void k_features(LearnedArgs a) {
#pragma clang fp contract(off)
    u32 n = a.counters[C_CAND];
    if (n > a.cap) n = a.cap;
    double Q = 0.0;
    for (int f = 0; f < 20; ++f) Q += a.qabs[f];
    const u64 stride = (u64)gridDim.x * blockDim.x;
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const u64 pr = a.cand[i];
        const u32 t = (u32)(pr >> 32), s = (u32)(pr & 0xffffffffu);
        const NodeMac mt = a.mac[t], ms = a.mac[s];
        const double dx = mt.cx - ms.cx, dy = mt.cy - ms.cy, dz = mt.cz - ms.cz;
        const double R = sqrt((dx * dx + dy * dy) + dz * dz);
        const i32 nt = a.ncnt[t], ns = a.ncnt[s];
        float f[16];
        f[0] = nt > a.n_crit ? 1.f : 0.f;
        f[1] = ns > a.n_crit ? 1.f : 0.f;
        f[2] = (float)level_of_offset_table(a.level_off_tab, a.L, t) / 8.f;
        f[3] = (float)level_of_offset_table(a.level_off_tab, a.L, s) / 8.f;
        f[4] = (float)(mt.r / R);
        f[5] = (float)(ms.r / R);
        f[6] = (float)((mt.r + ms.r) / R);
        f[7] = -lg10(R) / 2.f;
        const double qs = a.qabs[s], qt = a.qabs[t];
        f[8] = lg10(Q > 0 ? qs / Q : 0.0) / 8.f + 1.f;
        f[9] = qs > 0 ? (float)(fabs(a.qsum[s]) / qs) : 0.f;
        f[10] = 0.f;
        if (ns > a.n_crit && qs > 0) {
            const Prox* w4 = a.prox + (size_t)a.slot[s] * a.NPT;  // class 0 = degree 4
            double l1 = 0.0;
            for (int m = 0; m < 15; ++m) l1 += fabs(w4[m].w);
            f[10] = lg10(l1 / qs) / 2.f;
        }
        f[11] = lg10(Q > 0 ? qt / Q : 0.0) / 8.f + 1.f;
        for (int k = 12; k < 16; ++k) f[k] = 0.f;
        u32 packed[8];
        for (int k = 0; k < 8; ++k) packed[k] = (u32)f2bf(f[2 * k]) | ((u32)f2bf(f[2 * k + 1]) << 16);
        uint4* dst = reinterpret_cast<uint4*>(a.feat + (size_t)i * 16);
        dst[0] = make_uint4(packed[0], packed[1], packed[2], packed[3]);
        dst[1] = make_uint4(packed[4], packed[5], packed[6], packed[7]);
    }
}

// exclusive prefix of v over the 256 threads of the block, *total = sum
__device__ __forceinline__ u32 scan256(u32 v, u32* wsum, u32* total) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    u32 incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        const u32 t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    u32 b = 0, tot = 0;
    for (int k = 0; k < 4; ++k) {
        const u32 x = wsum[k];
        if (k < w) b += x;
        tot += x;
    }
    *total = tot;
    return b + incl - v;
}

// Accepted candidates (o0 > 0; degree class = number of positive ordinal
// logits) become list entries; the others go to the fallback frontier.
// Slots come from one atomic per list per 256 candidates.
__global__ __launch_bounds__(256) void k_resolve(LearnedArgs a, int use_model) {
    __shared__ u32 wsum[3][4];
    __shared__ u32 bases[3];
    u32 n = a.counters[C_CAND];
    if (n > a.cap) n = a.cap;
    const int tid = threadIdx.x;
    bool overflow = false;
    for (u64 b0 = (u64)blockIdx.x * 256; b0 < n; b0 += (u64)gridDim.x * 256) {
        const u64 i = b0 + tid;
        const bool ok = i < n;
        u64 pr = 0;
        bool acc = false;
        u32 dc = 0;
        int kind = 0;
        if (ok) {
            pr = a.cand[i];
            const u32 t = (u32)(pr >> 32), s = (u32)(pr & 0xffffffffu);
            kind = (a.ncnt[t] > a.n_crit ? 2 : 0) + (a.ncnt[s] > a.n_crit ? 1 : 0);
            if (use_model) {
                const float4 o = *reinterpret_cast<const float4*>(a.out + i * 4);
                acc = o.x > 0.f;
                dc = (o.y > 0.f ? 1u : 0u) + (o.z > 0.f ? 1u : 0u) + (o.w > 0.f ? 1u : 0u);
            }
        }
        const bool to_t = ok && acc && kind == 1;
        const bool to_n = ok && acc && kind >= 2;
        const bool to_f = ok && !acc;
        u32 tt, tn, tf;
        const u32 pt = scan256(to_t ? 1u : 0u, wsum[0], &tt);
        const u32 pn = scan256(to_n ? 1u : 0u, wsum[1], &tn);
        const u32 pf = scan256(to_f ? 1u : 0u, wsum[2], &tf);
        if (tid == 0) {
            bases[0] = tt ? atomicAdd(&a.counters[C_TLIST], tt) : 0u;
            bases[1] = tn ? atomicAdd(&a.counters[C_NLIST], tn) : 0u;
            bases[2] = tf ? atomicAdd(&a.counters[C_FRONT2], tf) : 0u;
        }
        __syncthreads();
        const u64 t = pr >> 32, s = pr & 0xffffffffu;
        const u64 key = (t << (a.W + 1 + a.DB)) | ((u64)dc << (a.W + 1)) | ((u64)(kind & 1) << a.W) | s;
        if (to_t) {
            const u32 st = bases[0] + pt;
            if (st < a.cap) a.tlist[st] = key;
            else overflow = true;
        }
        if (to_n) {
            const u32 sn = bases[1] + pn;
            if (sn < a.cap) a.nlist[sn] = key;
            else overflow = true;
        }
        if (to_f) {
            const u32 sf = bases[2] + pf;
            if (sf < a.cap) a.front[sf] = pr;
            else overflow = true;
        }
        __syncthreads();  // wsum / bases reused by the next round
    }
    if (overflow) atomicOr(&a.counters[C_OVERFLOW], 1u);
}

// one FP64 kernel evaluation q (y - x) / den added to acc
__device__ __forceinline__ void kern64(double x0, double x1, double x2, double y0, double y1, double y2, double q,
                                       int dist2, double* acc) {
    const double d0 = y0 - x0, d1 = y1 - x1, d2 = y2 - x2;
    const double den = dist2 ? 0.5 * ((d0 * d0 + d1 * d1) + d2 * d2) : 1.0 - ((x0 * y0 + x1 * y1) + x2 * y2);
    const double w = q / den;
    acc[0] += w * d0;
    acc[1] += w * d1;
    acc[2] += w * d2;
}

// Label generator: for every candidate (t, s) and degree class c, the
// largest error over t's particles of the interaction the pair would get at
// that degree -- PC (source proxies), CP (interpolation from the target's
// points) or CC (both) -- against the exact sum over s's particles; FP64.
// One workgroup per candidate.
__global__ __launch_bounds__(256) void k_pair_errors(LearnedArgs la, EvalArgs a, int dist2, u32 lim,
                                                      double* __restrict__ err) {
    __shared__ double al[kMaxNp * 4][3];   // target coefficients of every class (CP / CC)
    __shared__ double wt[kMaxNp][3];
    __shared__ double nd[kMaxNp];
    __shared__ double red[3 * 256];
    __shared__ double emax[4][256];
    u32 n = la.counters[C_CAND];
    if (n > la.cap) n = la.cap;
    if (n > lim) n = lim;
    const int tid = threadIdx.x;
    for (u32 ci = blockIdx.x; ci < n; ci += gridDim.x) {
        const u64 pr = la.cand[ci];
        const u32 t = (u32)(pr >> 32), s = (u32)(pr & 0xffffffffu);
        const i32 tb = a.nbeg[t], te = a.nend[t], sb = a.nbeg[s], se = a.nend[s];
        const bool big_t = te - tb > a.n_crit, big_s = se - sb > a.n_crit;
        const NodeGeo& gt = a.geo[t];
        // target side: coefficients alpha_c = V^{-1} (W at the target's class-c points)
        if (big_t) {
            for (int c = 0; c < a.ndeg; ++c) {
                const int np = STC_PICK4(a.cls.np, c), d = STC_PICK4(a.cls.deg, c);
                const int poff = STC_PICK4(a.cls.poff, c), qoff = STC_PICK4(a.cls.qoff, c);
                const int S = 256 / np;
                const int m = tid % np, sl = tid / np;
                double acc[3] = {0.0, 0.0, 0.0};
                if (sl < S) {
                    double y[3];
                    const double nrm = proxy_point(gt, a.ref.points + 3 * (poff + m), y);
                    if (sl == 0) nd[m] = ipow(nrm, d);
                    if (big_s) {
                        const Prox* ps = a.prox + (size_t)a.slot[s] * a.NPT + poff;
                        for (int k = sl; k < np; k += S) kern64(y[0], y[1], y[2], ps[k].x, ps[k].y, ps[k].z, ps[k].w, dist2, acc);
                    } else {
                        for (i32 j = sb + sl; j < se; j += S) kern64(y[0], y[1], y[2], a.sx[j], a.sy[j], a.sz[j], a.sq[j], dist2, acc);
                    }
                }
                for (int k = 0; k < 3; ++k) red[k * 256 + tid] = sl < S ? acc[k] : 0.0;
                __syncthreads();
                if (tid < np) {
                    for (int k = 0; k < 3; ++k) {
                        double v = 0.0;
                        for (int q = 0; q < S; ++q) v += red[k * 256 + q * np + tid];
                        wt[tid][k] = v;
                    }
                }
                __syncthreads();
                block_matvec<256, 3>(a.ref.vinvT + qoff, np, np, nd, wt, red, &al[poff]);
            }
        }
        double e[4] = {0.0, 0.0, 0.0, 0.0};
        for (i32 i0 = tb; i0 < te; i0 += 256) {
            const i32 i = i0 + tid;
            if (i < te) {
                const double x0 = a.sx[i], x1 = a.sy[i], x2 = a.sz[i];
                double ex[3] = {0.0, 0.0, 0.0};
                for (i32 j = sb; j < se; ++j) kern64(x0, x1, x2, a.sx[j], a.sy[j], a.sz[j], a.sq[j], dist2, ex);
                for (int c = 0; c < a.ndeg; ++c) {
                    const int np = STC_PICK4(a.cls.np, c), d = STC_PICK4(a.cls.deg, c);
                    const int poff = STC_PICK4(a.cls.poff, c);
                    double ap[3] = {0.0, 0.0, 0.0};
                    if (!big_t) {  // PC: the source's proxy points
                        const Prox* ps = a.prox + (size_t)a.slot[s] * a.NPT + poff;
                        for (int k = 0; k < np; ++k) kern64(x0, x1, x2, ps[k].x, ps[k].y, ps[k].z, ps[k].w, dist2, ap);
                    } else {       // CP / CC: interpolate the target's coefficients at x_i
                        double P[3][kMaxDegree + 1];
                        for (int cc = 0; cc < 3; ++cc) {
                            const double be = (gt.minv[cc][0] * x0 + gt.minv[cc][1] * x1) + gt.minv[cc][2] * x2;
                            P[cc][0] = 1.0;
                            for (int k = 1; k <= d; ++k) P[cc][k] = P[cc][k - 1] * be;
                        }
                        for (int k = 0; k < np; ++k) {
                            const int* ex3 = a.ref.expo + 3 * (poff + k);
                            const double B = a.ref.coef[poff + k] * (P[0][ex3[0]] * P[1][ex3[1]] * P[2][ex3[2]]);
                            ap[0] += B * al[poff + k][0];
                            ap[1] += B * al[poff + k][1];
                            ap[2] += B * al[poff + k][2];
                        }
                    }
                    const double d0 = ap[0] - ex[0], d1 = ap[1] - ex[1], d2 = ap[2] - ex[2];
                    const double en = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
                    e[c] = en > e[c] ? en : e[c];
                }
            }
        }
        for (int c = 0; c < 4; ++c) emax[c][tid] = e[c];
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (tid < h)
                for (int c = 0; c < 4; ++c) emax[c][tid] = emax[c][tid + h] > emax[c][tid] ? emax[c][tid + h] : emax[c][tid];
            __syncthreads();
        }
        if (tid < 4) err[(size_t)ci * 4 + tid] = tid < a.ndeg ? emax[tid][0] : 0.0;
        __syncthreads();
    }
}

// Labels from the errors: accept iff some class meets tol; the ordinal
// targets say whether the smallest such class lies above class k (k = 0..2).
__global__ __launch_bounds__(256) void k_labels(const u32* __restrict__ d_n, u32 cap, u32 lim,
                                                 const double* __restrict__ err, double tol, float* __restrict__ y) {
    u32 n = *d_n;
    if (n > cap) n = cap;
    if (n > lim) n = lim;
    const u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int cmin = 4;
    for (int c = 3; c >= 0; --c)
        if (err[i * 4 + c] <= tol) cmin = c;
    float4 v;
    v.x = cmin < 4 ? 1.f : 0.f;
    v.y = cmin < 4 && cmin > 0 ? 1.f : 0.f;
    v.z = cmin < 4 && cmin > 1 ? 1.f : 0.f;
    v.w = cmin < 4 && cmin > 2 ? 1.f : 0.f;
    *reinterpret_cast<float4*>(y + i * 4) = v;
}

}  // namespace

void launch_pair_errors(hipStream_t s, const LearnedArgs& la, const EvalArgs& a, int dist2, u32 lim, double* err) {
    hipLaunchKernelGGL(k_pair_errors, dim3(2048), dim3(256), 0, s, la, a, dist2, lim, err);
}

void launch_labels(hipStream_t s, const LearnedArgs& la, u32 lim, const double* err, double tol, float* y) {
    const u32 m = std::min(la.cap, lim);
    if (m == 0) return;
    hipLaunchKernelGGL(k_labels, dim3((m + 255) / 256), dim3(256), 0, s, la.counters + C_CAND, la.cap, lim, err, tol,
                       y);
}

void launch_node_charge_sums(hipStream_t s, const i32* nbeg, const i32* nend, const i64* level_off_host, int L,
                             const double* q, double* qabs, double* qsum) {
    for (int lvl = L; lvl >= 0; --lvl) {
        const i64 node0 = level_off_host[lvl], nn = level_off_host[lvl + 1] - node0;
        const i64 child_off = lvl < L ? level_off_host[lvl + 1] : 0;
        hipLaunchKernelGGL(k_qsum_level, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, node0, nn, lvl, L,
                           child_off, nbeg, nend, q, qabs, qsum);
    }
}

void launch_features(hipStream_t s, const LearnedArgs& a) {
    hipLaunchKernelGGL(k_features, dim3(1024), dim3(256), 0, s, a);
}

void launch_mlp_forward_list(hipStream_t s, const LearnedArgs& a) {
    launch_mlp_forward(s, a.feat, 0, a.counters + C_CAND, a.cap, a.model, a.out);
}

void launch_resolve(hipStream_t s, const LearnedArgs& a, bool use_model) {
    hipLaunchKernelGGL(k_resolve, dim3(1024), dim3(256), 0, s, a, use_model ? 1 : 0);
}

// 4 pi sqrt(mean |u_i|^2): the size of W (the sum the cross product with x
// turns into u), the unit in which label tolerances are given.  One
// workgroup: strided FP64 sums per thread, then a fixed-order tree.
__global__ __launch_bounds__(256) void k_label_scale(const double* __restrict__ u, i64 n, double* __restrict__ out) {
    __shared__ double red[256];
    double acc = 0.0;
    for (i64 i = threadIdx.x; i < n; i += 256) {
        const double a = u[3 * i], b = u[3 * i + 1], c = u[3 * i + 2];
        acc += (a * a + b * b) + c * c;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = n > 0 ? 4.0 * 3.141592653589793 * sqrt(red[0] / (double)n) : 0.0;
}

void launch_label_scale(hipStream_t s, const double* u, i64 n, double* out) {
    hipLaunchKernelGGL(k_label_scale, dim3(1), dim3(256), 0, s, u, n, out);
}

}  // namespace stc
