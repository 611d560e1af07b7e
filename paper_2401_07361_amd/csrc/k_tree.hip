// Tree build, upward pass and dual tree traversal kernels.
#include "common.hpp"
#include "kernels.hpp"

namespace stc {

// ---------------------------------------------------------------------------
// Point location (Sec. 3, the triangle tree).  Root face: the lowest face
// index whose three edge orientations are all >= 0.  Inside a triangle the
// centre child's vertices (m12, m23, m31) are read from the next level; the
// point goes to corner 1, 2 or 3 if it lies strictly outside the centre child
// across the edge facing that corner (tested in that order), otherwise to
// the centre child.  All orientations are exact.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bin(const double* __restrict__ x, i64 n,
                                              const NodeGeo* __restrict__ geo, int L,
                                              u64* __restrict__ keys, u32* __restrict__ flags) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double p[3] = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
    int face = -1;
    for (int f = 0; f < 20 && face < 0; ++f) {
        const NodeGeo& g = geo[f];
        if (orient(g.v[0], g.v[1], p) >= 0 && orient(g.v[1], g.v[2], p) >= 0 &&
            orient(g.v[2], g.v[0], p) >= 0)
            face = f;
    }
    if (face < 0) {  // non-finite input: no face contains it
        atomicOr(&flags[0], 1u);
        face = 0;
    }
    u32 key = (u32)face;
    i64 off = 20;  // level_offset(1)
    for (int lvl = 0; lvl < L; ++lvl) {
        const NodeGeo& c = geo[off + 4 * (i64)key + 3];  // (m12, m23, m31)
        u32 digit;
        if (orient(c.v[2], c.v[0], p) < 0) digit = 0;
        else if (orient(c.v[0], c.v[1], p) < 0) digit = 1;
        else if (orient(c.v[1], c.v[2], p) < 0) digit = 2;
        else digit = 3;
        key = 4 * key + digit;
        off = 4 * off + 20;  // level_offset(lvl + 2)
    }
    keys[i] = ((u64)key << 32) | (u64)i;
}

// sorted position -> input index, leaf key, FP64 SoA positions
__global__ __launch_bounds__(256) void k_gather(const u64* __restrict__ keys, i64 n,
                                                 const double* __restrict__ x, i32* __restrict__ perm,
                                                 u32* __restrict__ leaf, double* __restrict__ sx,
                                                 double* __restrict__ sy, double* __restrict__ sz) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const u64 k = keys[i];
    const u32 idx = (u32)(k & 0xffffffffu);
    perm[i] = (i32)idx;
    leaf[i] = (u32)(k >> 32);
    sx[i] = x[3 * (i64)idx];
    sy[i] = x[3 * (i64)idx + 1];
    sz[i] = x[3 * (i64)idx + 2];
}

// Particle range [begin, end) of every node that holds particles, from the
// boundaries of the sorted leaf keys at each level.  Arrays must be zeroed.
__global__ __launch_bounds__(256) void k_node_ranges(const u32* __restrict__ leaf, i64 n, int L,
                                                      i32* __restrict__ nbeg, i32* __restrict__ nend) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const u32 k = leaf[i];
    const u32 kp = i > 0 ? leaf[i - 1] : 0u;
    const u32 kn = i + 1 < n ? leaf[i + 1] : 0u;
    i64 off = 0;
    for (int lvl = 0; lvl <= L; ++lvl) {
        const int sh = 2 * (L - lvl);
        const u32 pf = k >> sh;
        if (i == 0 || (kp >> sh) != pf) nbeg[off + pf] = (i32)i;
        if (i == n - 1 || (kn >> sh) != pf) nend[off + pf] = (i32)(i + 1);
        off = 4 * off + 20;
    }
}

__global__ __launch_bounds__(256) void k_charges(const i32* __restrict__ perm, i64 n,
                                                  const double* __restrict__ zeta,
                                                  const double* __restrict__ area, double* __restrict__ q) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const i32 j = perm[i];
    q[i] = zeta[j] * area[j];
}

// ---------------------------------------------------------------------------
// Upward pass (Sec. 3, particle-cluster interaction): for every node with
// more than N_T particles, omega_k = sum_j B_k(b(y_j)) q_j with b = M^{-1} y
// and the multinomial-scaled SBB basis, then the proxy charges
//   w_m = |b_m1 v1 + b_m2 v2 + b_m3 v3|^d * sum_k (V_ref^{-1})_{km} omega_k,
// i.e. w = V^{-T} omega for the node's Vandermonde matrix V = diag(s^d) V_ref.
// One workgroup per node; chunks of 64 particles have their barycentric
// powers staged in LDS, and thread t accumulates basis function t % np over
// every (256 / np)-th particle of the chunk.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_p2m(const i32* __restrict__ nbeg, const i32* __restrict__ nend,
                                              i64 n_nodes, int n_crit, const NodeGeo* __restrict__ geo,
                                              const double* __restrict__ sx, const double* __restrict__ sy,
                                              const double* __restrict__ sz, const double* __restrict__ q,
                                              RefDev ref, double* __restrict__ w) {
    __shared__ double pw[64][3][kMaxDegree + 1];
    __shared__ double qs[64];
    __shared__ double red[256];
    __shared__ double omega[kMaxNp];
    const int tid = threadIdx.x;
    const int d = ref.degree, np = ref.np;
    const int S = 256 / np;  // particle slices
    const int k = tid % np, sl = tid / np;
    int e0 = 0, e1 = 0, e2 = 0;
    if (sl < S) {
        e0 = ref.expo[3 * k];
        e1 = ref.expo[3 * k + 1];
        e2 = ref.expo[3 * k + 2];
    }
    for (i64 node = blockIdx.x; node < n_nodes; node += gridDim.x) {
        const i32 b = nbeg[node], e = nend[node];
        if (e - b <= n_crit) continue;  // uniform over the block
        const NodeGeo& g = geo[node];
        double acc = 0.0;
        for (i32 c0 = b; c0 < e; c0 += 64) {
            const int cnt = (e - c0) < 64 ? (e - c0) : 64;
            if (tid < cnt) {
                const i32 j = c0 + tid;
                const double y0 = sx[j], y1 = sy[j], y2 = sz[j];
                for (int a = 0; a < 3; ++a) {
                    const double be = (g.minv[a][0] * y0 + g.minv[a][1] * y1) + g.minv[a][2] * y2;
                    double pp = 1.0;
                    for (int t = 0; t <= d; ++t) {
                        pw[tid][a][t] = pp;
                        pp *= be;
                    }
                }
                qs[tid] = q[j];
            }
            __syncthreads();
            if (sl < S) {
                for (int j = sl; j < cnt; j += S) acc += qs[j] * (pw[j][0][e0] * pw[j][1][e1] * pw[j][2][e2]);
            }
            __syncthreads();
        }
        red[tid] = (sl < S) ? acc : 0.0;
        __syncthreads();
        if (tid < np) {
            double s = 0.0;
            for (int t = 0; t < S; ++t) s += red[t * np + tid];
            omega[tid] = ref.coef[tid] * s;
        }
        __syncthreads();
        for (int m = tid; m < np; m += 256) {
            double y[3];
            const double nrm = proxy_point(g, ref.points + 3 * m, y);
            double s = 0.0;
            for (int kk = 0; kk < np; ++kk) s += ref.vinv[(size_t)kk * np + m] * omega[kk];
            w[(size_t)node * np + m] = ipow(nrm, d) * s;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Dual tree traversal (Sec. 3), level-synchronous.  Iteration k reads the
// frontier of node pairs and, per pair (t, s):
//   well separated: (r_t + r_s)^2 < theta^2 R^2 (FP64, no contraction) ->
//     PP / PC / CP / CC by which side has more than N_T particles;
//   else both small -> PP;
//   else split the side with more particles (tie: target), or the other one
//     if it cannot be split, or emit PP if neither can;
//   splitting pushes the non-empty children into the next frontier.
// Target-particle entries (PP, PC) and target-proxy entries (CP, CC) go to
// two lists as sort keys (t << (W+1)) | (type << W) | s.
// ---------------------------------------------------------------------------
__global__ void k_trav_init(const i32* __restrict__ nbeg, const i32* __restrict__ nend,
                            u64* __restrict__ front, u32 cap, u32* __restrict__ counters) {
    const int i = threadIdx.x;  // 512 threads, 400 used
    const bool ok = i < 400 && (nend[i / 20] - nbeg[i / 20]) > 0 && (nend[i % 20] - nbeg[i % 20]) > 0;
    const u32 slot = wave_append(&counters[C_FRONT], ok);
    if (ok) {
        if (slot < cap) front[slot] = ((u64)(i / 20) << 32) | (u64)(i % 20);
        else atomicOr(&counters[C_OVERFLOW], 1u);
    }
}

__device__ __forceinline__ bool mac_separated(const NodeGeo& a, const NodeGeo& b, double theta2) {
#pragma clang fp contract(off)
    const double s = a.r + b.r;
    const double dx = a.c[0] - b.c[0];
    const double dy = a.c[1] - b.c[1];
    const double dz = a.c[2] - b.c[2];
    const double R2 = (dx * dx + dy * dy) + dz * dz;
    return s * s < theta2 * R2;
}

__global__ __launch_bounds__(256) void k_trav_level(
    int iter, const u64* __restrict__ fin, u64* __restrict__ fout, u32 cap, const i32* __restrict__ nbeg,
    const i32* __restrict__ nend, const i64* __restrict__ level_off_tab, int L, const NodeGeo* __restrict__ geo,
    double theta2, int n_crit, int W, u64* __restrict__ tlist, u64* __restrict__ nlist, u32* __restrict__ counters) {
    u32 nin = counters[C_FRONT + iter];
    if (nin > cap) nin = cap;
    const int lane = threadIdx.x & 63;
    const u64 stride = (u64)gridDim.x * blockDim.x;
    // every lane of a wave runs the same number of iterations (ballots below)
    for (u64 base = (u64)blockIdx.x * blockDim.x + (threadIdx.x - lane); base < nin; base += stride) {
        const u64 i = base + lane;
        const bool active = i < nin;
        int kind = -1;        // 0 PP, 1 PC, 2 CP, 3 CC; -1 none
        bool split_t = false; // when children are pushed: which side was split
        int nkids = 0;
        u32 kid_ids[4] = {0, 0, 0, 0};
        u32 t = 0, s = 0;
        if (active) {
            const u64 pr = fin[i];
            t = (u32)(pr >> 32);
            s = (u32)(pr & 0xffffffffu);
            const i32 nt = nend[t] - nbeg[t], ns = nend[s] - nbeg[s];
            const bool big_t = nt > n_crit, big_s = ns > n_crit;
            if (mac_separated(geo[t], geo[s], theta2)) {
                kind = (big_t ? 2 : 0) + (big_s ? 1 : 0);
            } else if (!big_t && !big_s) {
                kind = 0;
            } else {
                const int lt = level_of_offset_table(level_off_tab, L, t);
                const int ls = level_of_offset_table(level_off_tab, L, s);
                const bool int_t = big_t && lt < L, int_s = big_s && ls < L;
                split_t = nt >= ns;
                if (split_t && !int_t) split_t = false;
                if (!split_t && !int_s) {
                    if (int_t) split_t = true;
                    else kind = 0;
                }
                if (kind < 0) {
                    const u32 x = split_t ? t : s;
                    const int lx = split_t ? lt : ls;
                    const i64 child0 = level_off_tab[lx + 1] + 4 * ((i64)x - level_off_tab[lx]);
                    for (int c = 0; c < 4; ++c) {
                        const u32 cid = (u32)(child0 + c);
                        if (nend[cid] - nbeg[cid] > 0) kid_ids[nkids++] = cid;
                    }
                }
            }
        }
        // list appends (PP/PC -> tlist, CP/CC -> nlist)
        const bool to_t = kind == 0 || kind == 1;
        const bool to_n = kind == 2 || kind == 3;
        const u32 st = wave_append(&counters[C_TLIST], to_t);
        const u32 sn = wave_append(&counters[C_NLIST], to_n);
        const u64 keyv = ((u64)t << (W + 1)) | ((u64)(kind & 1) << W) | (u64)s;
        if (to_t) {
            if (st < cap) tlist[st] = keyv;
            else atomicOr(&counters[C_OVERFLOW], 1u);
        }
        if (to_n) {
            if (sn < cap) nlist[sn] = keyv;
            else atomicOr(&counters[C_OVERFLOW], 1u);
        }
        // frontier pushes: wave inclusive scan of nkids
        int incl = nkids;
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(incl, o, 64);
            if (lane >= o) incl += v;
        }
        const int total = __shfl(incl, 63, 64);
        if (total > 0) {
            u32 fbase = 0;
            if (lane == 0) fbase = atomicAdd(&counters[C_FRONT + iter + 1], (u32)total);
            fbase = __shfl(fbase, 0, 64);
            const u32 my = fbase + (u32)(incl - nkids);
            for (int c = 0; c < nkids; ++c) {
                const u64 pr = split_t ? (((u64)kid_ids[c] << 32) | (u64)s) : (((u64)t << 32) | (u64)kid_ids[c]);
                if (my + c < cap) fout[my + c] = pr;
                else atomicOr(&counters[C_OVERFLOW], 1u);
            }
        }
    }
}

// Segments of a sorted list: entries with the same target t occupy
// [seg_beg[t], seg_end[t]).  Arrays must be zeroed before.
__global__ __launch_bounds__(256) void k_segments(const u64* __restrict__ list, const u32* __restrict__ d_n,
                                                   u32 cap, int W, i32* __restrict__ seg_beg,
                                                   i32* __restrict__ seg_end) {
    u32 n = *d_n;
    if (n > cap) n = cap;
    const u64 stride = (u64)gridDim.x * blockDim.x;
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const u64 t = list[i] >> (W + 1);
        if (i == 0 || (list[i - 1] >> (W + 1)) != t) seg_beg[t] = (i32)i;
        if (i + 1 == n || (list[i + 1] >> (W + 1)) != t) seg_end[t] = (i32)(i + 1);
    }
}

__global__ __launch_bounds__(256) void k_fill_u32(u32* __restrict__ p, i64 n, u32 v) {
    const u64 stride = (u64)gridDim.x * blockDim.x;
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < (u64)n; i += stride) p[i] = v;
}

__global__ __launch_bounds__(256) void k_fill_f64(double* __restrict__ p, i64 n, double v) {
    const u64 stride = (u64)gridDim.x * blockDim.x;
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < (u64)n; i += stride) p[i] = v;
}

// Kernel-evaluation count implied by the lists (introspection only).
__global__ __launch_bounds__(256) void k_count_evals(const u64* __restrict__ list, const u32* __restrict__ d_n,
                                                      u32 cap, int W, int np, const i32* __restrict__ nbeg,
                                                      const i32* __restrict__ nend, int target_is_proxy,
                                                      unsigned long long* __restrict__ out) {
    // out[0], out[1]: evaluations of type 0 / 1 entries; out[2], out[3]: entries
    u32 n = *d_n;
    if (n > cap) n = cap;
    const u64 stride = (u64)gridDim.x * blockDim.x;
    const u64 mask = ((u64)1 << W) - 1;
    unsigned long long a0 = 0, a1 = 0, c0 = 0, c1 = 0;
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const u64 k = list[i];
        const u64 t = k >> (W + 1), s = k & mask;
        const int ty = (int)((k >> W) & 1);
        const u64 nt = target_is_proxy ? (u64)np : (u64)(nend[t] - nbeg[t]);
        const u64 ns = ty ? (u64)np : (u64)(nend[s] - nbeg[s]);
        u64 v = nt * ns;
        if (!target_is_proxy && !ty && t == s) v -= nt;
        if (ty) { a1 += v; c1 += 1; }
        else { a0 += v; c0 += 1; }
    }
    atomicAdd(&out[0], a0);
    atomicAdd(&out[1], a1);
    atomicAdd(&out[2], c0);
    atomicAdd(&out[3], c1);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {
inline unsigned blocks_for(i64 n, int threads) { return (unsigned)((n + threads - 1) / threads); }
}

void launch_bin(hipStream_t s, const double* x, i64 n, const NodeGeo* geo, int L, u64* keys, u32* flags) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_bin, dim3(blocks_for(n, 256)), dim3(256), 0, s, x, n, geo, L, keys, flags);
}

void launch_gather(hipStream_t s, const u64* keys, i64 n, const double* x, i32* perm, u32* leaf, double* sx,
                   double* sy, double* sz) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather, dim3(blocks_for(n, 256)), dim3(256), 0, s, keys, n, x, perm, leaf, sx, sy, sz);
}

void launch_node_ranges(hipStream_t s, const u32* leaf, i64 n, int L, i32* nbeg, i32* nend) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_node_ranges, dim3(blocks_for(n, 256)), dim3(256), 0, s, leaf, n, L, nbeg, nend);
}

void launch_charges(hipStream_t s, const i32* perm, i64 n, const double* zeta, const double* area, double* q) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_charges, dim3(blocks_for(n, 256)), dim3(256), 0, s, perm, n, zeta, area, q);
}

void launch_p2m(hipStream_t s, const i32* nbeg, const i32* nend, i64 n_nodes, int n_crit, const NodeGeo* geo,
                const double* sx, const double* sy, const double* sz, const double* q, RefDev ref, double* w) {
    const unsigned grid = (unsigned)(n_nodes < 8192 ? n_nodes : 8192);
    hipLaunchKernelGGL(k_p2m, dim3(grid), dim3(256), 0, s, nbeg, nend, n_nodes, n_crit, geo, sx, sy, sz, q, ref, w);
}

void launch_fill_u32(hipStream_t s, u32* p, i64 n, u32 v) {
    if (n <= 0) return;
    const i64 b = blocks_for(n, 256);
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)(b < 4096 ? b : 4096)), dim3(256), 0, s, p, n, v);
}

void launch_fill_f64(hipStream_t s, double* p, i64 n, double v) {
    if (n <= 0) return;
    const i64 b = blocks_for(n, 256);
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)(b < 4096 ? b : 4096)), dim3(256), 0, s, p, n, v);
}

void launch_traverse(hipStream_t s, const i32* nbeg, const i32* nend, const i64* level_off_tab, int L,
                     const NodeGeo* geo, double theta, int n_crit, int W, u64* front0, u64* front1, u32 cap,
                     u64* tlist, u64* nlist, u32* counters) {
    launch_fill_u32(s, counters, C_COUNT, 0u);
    hipLaunchKernelGGL(k_trav_init, dim3(1), dim3(512), 0, s, nbeg, nend, front0, cap, counters);
    const double theta2 = theta * theta;
    const int iters = 2 * L + 2;
    for (int it = 0; it < iters; ++it) {
        const u64* fin = (it % 2 == 0) ? front0 : front1;
        u64* fout = (it % 2 == 0) ? front1 : front0;
        hipLaunchKernelGGL(k_trav_level, dim3(1024), dim3(256), 0, s, it, fin, fout, cap, nbeg, nend,
                           level_off_tab, L, geo, theta2, n_crit, W, tlist, nlist, counters);
    }
}

void launch_segments(hipStream_t s, const u64* list, const u32* d_n, u32 cap, int W, i32* seg_beg, i32* seg_end) {
    hipLaunchKernelGGL(k_segments, dim3(1024), dim3(256), 0, s, list, d_n, cap, W, seg_beg, seg_end);
}

void launch_count_evals(hipStream_t s, const u64* list, const u32* d_n, u32 cap, int W, int np, const i32* nbeg,
                        const i32* nend, int target_is_proxy, unsigned long long* out) {
    hipLaunchKernelGGL(k_count_evals, dim3(256), dim3(256), 0, s, list, d_n, cap, W, np, nbeg, nend,
                       target_is_proxy, out);
}

}  // namespace stc
