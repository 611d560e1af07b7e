// Tree build, upward pass and dual tree traversal kernels.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace stc {

// ---------------------------------------------------------------------------
// Point location (Sec. 3, the triangle tree).  Root face: the lowest face
// index whose three edge orientations are all >= 0.  Inside a triangle the
// centre child's vertices (m12, m23, m31) are read from the next level; the
// point goes to corner 1, 2 or 3 if it lies strictly outside the centre child
// across the edge facing that corner (tested in that order), otherwise to
// the centre child.  All orientations are exact.  The sort key is
// (member, leaf key, index): the member of particle i is the last m with
// off[m] <= i (a fixed-index scan, so the offsets stay in kernel arguments).
//
// Two passes: k_bin decides every orientation with the FP64 filter or the
// double-double stage and queues the points where neither can (an exact zero
// that no structural test recognises); k_bin_exact locates the queued points
// with the exact expansion.  Keeping the expansion out of k_bin keeps its register
// count, and so its occupancy, those of the common path.
// ---------------------------------------------------------------------------
template <bool EXACT>
__device__ __forceinline__ int orient_sel(const double* a, const double* b, const double* p, double pb) {
    if (EXACT) return orient(a, b, p, pb);
    return orient_filtered(a, b, p, pb);  // -2 where only the exact expansion can decide
}

// Leaf key of point p (face in the top bits, one base-4 digit per level).
// Returns false if, without EXACT, an orientation could not be decided.
template <bool EXACT>
__device__ __forceinline__ bool locate(const double* p, const NodeGeo* __restrict__ geo, int L, u32* key_out) {
    const double pb = perm_bound(p);
    // candidate: the face whose circumcentre is nearest; if p is strictly
    // inside it no other face contains p, else scan in index order
    int best = 0;
    double bd = -2.0;
    for (int f = 0; f < 20; ++f) {
        const double dt = (geo[f].c[0] * p[0] + geo[f].c[1] * p[1]) + geo[f].c[2] * p[2];
        if (dt > bd) {
            bd = dt;
            best = f;
        }
    }
    int face = -1;
    {
        const NodeGeo& g = geo[best];
        int o = orient_sel<EXACT>(g.v[0], g.v[1], p, pb);
        if (o == -2) return false;
        if (o > 0) {
            o = orient_sel<EXACT>(g.v[1], g.v[2], p, pb);
            if (o == -2) return false;
            if (o > 0) {
                o = orient_sel<EXACT>(g.v[2], g.v[0], p, pb);
                if (o == -2) return false;
                if (o > 0) face = best;
            }
        }
    }
    for (int f = 0; f < 20 && face < 0; ++f) {
        const NodeGeo& g = geo[f];
        int o = orient_sel<EXACT>(g.v[0], g.v[1], p, pb);
        if (o == -2) return false;
        if (o < 0) continue;
        o = orient_sel<EXACT>(g.v[1], g.v[2], p, pb);
        if (o == -2) return false;
        if (o < 0) continue;
        o = orient_sel<EXACT>(g.v[2], g.v[0], p, pb);
        if (o == -2) return false;
        if (o < 0) continue;
        face = f;
    }
    if (face < 0) face = 0;  // cannot happen for a finite point (the faces cover the sphere)
    u32 key = (u32)face;
    i64 off = 20;  // level_offset(1)
    for (int lvl = 0; lvl < L; ++lvl) {
        const NodeGeo& c = geo[off + 4 * (i64)key + 3];  // (m12, m23, m31)
        u32 digit = 3;
        int o = orient_sel<EXACT>(c.v[2], c.v[0], p, pb);
        if (o == -2) return false;
        if (o < 0) digit = 0;
        else {
            o = orient_sel<EXACT>(c.v[0], c.v[1], p, pb);
            if (o == -2) return false;
            if (o < 0) digit = 1;
            else {
                o = orient_sel<EXACT>(c.v[1], c.v[2], p, pb);
                if (o == -2) return false;
                if (o < 0) digit = 2;
            }
        }
        key = 4 * key + digit;
        off = 4 * off + 20;  // level_offset(lvl + 2)
    }
    *key_out = key;
    return true;
}

__device__ __forceinline__ u64 bin_key(u32 key, i64 i, int L, const MemberOffsets& mo) {
    u32 member = 0;
    if (mo.m > 1) {
#pragma unroll
        for (int k = 1; k < kMaxMembers; ++k)
            if (k < mo.m && mo.off[k] <= i) member = (u32)k;
    }
    key |= member << (2 * L + 5);
    return ((u64)key << 32) | (u64)i;
}

// queue: room for n indices; flags[F_BIN_EXACT] counts the queued points
__global__ __launch_bounds__(256) void k_bin(const double* __restrict__ x, i64 n,
                                              const NodeGeo* __restrict__ geo, int L, MemberOffsets mo,
                                              u64* __restrict__ keys, u32* __restrict__ queue,
                                              u32* __restrict__ flags) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double p[3] = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
    u32 key = 0;
    bool decided = true;
    if (!(isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]))) {
        atomicOr(&flags[F_NONFINITE], 1u);  // reported at synchronisation; the key is arbitrary
    } else {
        decided = locate<false>(p, geo, L, &key);
    }
    const u32 slot = wave_append(&flags[F_BIN_EXACT], !decided);
    if (decided) keys[i] = bin_key(key, i, L, mo);
    else queue[slot] = (u32)i;
}

__global__ __launch_bounds__(256) void k_bin_exact(const double* __restrict__ x, const NodeGeo* __restrict__ geo,
                                                    int L, MemberOffsets mo, const u32* __restrict__ queue,
                                                    const u32* __restrict__ flags, u64* __restrict__ keys) {
    const u32 cnt = flags[F_BIN_EXACT];
    for (u32 q = blockIdx.x * blockDim.x + threadIdx.x; q < cnt; q += gridDim.x * blockDim.x) {
        const i64 i = queue[q];
        const double p[3] = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
        u32 key = 0;
        (void)locate<true>(p, geo, L, &key);
        keys[i] = bin_key(key, i, L, mo);
    }
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
// boundaries of the sorted leaf keys at each level (the member bits above the
// key take part in the comparison).  Arrays must be zeroed.
__global__ __launch_bounds__(256) void k_node_ranges(const u32* __restrict__ leaf, i64 n, int L, int NB,
                                                      i32* __restrict__ nbeg, i32* __restrict__ nend) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int LB = 2 * L + 5;
    const u32 k = leaf[i];
    const u32 kp = i > 0 ? leaf[i - 1] : 0u;
    const u32 kn = i + 1 < n ? leaf[i + 1] : 0u;
    const i64 base = (i64)(k >> LB) << NB;
    const u32 kl = k & ((1u << LB) - 1u);
    i64 off = 0;
    for (int lvl = 0; lvl <= L; ++lvl) {
        const int sh = 2 * (L - lvl);
        const u32 pf = k >> sh;
        const i64 node = base + off + (kl >> sh);
        if (i == 0 || (kp >> sh) != pf) nbeg[node] = (i32)i;
        if (i == n - 1 || (kn >> sh) != pf) nend[node] = (i32)(i + 1);
        off = 4 * off + 20;
    }
}

// Ramp A(t) of the forcing (Sec. 4.4, polar vortex collapse): a half cosine up
// over [0, T_p), 1 until T_f - T_p, a half cosine down until T_f, 0 outside
// [0, T_f).  On the last piece (1 - cos(pi + a)) / 2 = (1 + cos a) / 2.
__device__ double forcing_ramp(double t, double tp, double tf) {
    constexpr double kPi = 3.141592653589793;
    if (!(t >= 0.0) || t >= tf) return 0.0;
    if (t < tp) return 0.5 * (1.0 - cos(t / tp * kPi));
    if (t < tf - tp) return 1.0;
    return 0.5 * (1.0 + cos((t - tf + tp) / tp * kPi));
}

// F_R / (amp A) at a point in any direction x (stage points of RK4 lie off the
// sphere): B(lat) cos(k lon) without trigonometric functions.  With rho the
// distance from the axis, tan^2(lat) = z^2 / rho^2, so the ratio
// r = tan^2(lat1) / tan^2(lat) = tan^2(lat1) rho^2 / z^2 and B = r e^(1 - r)
// for z > 0 (B = 0 for lat <= 0; B -> 0 at the pole, where r = 0).
// cos(k lon) = Re((x + i y)^k) / rho^k, from the unit vector (x, y) / rho.
__device__ double forcing_shape(int k, double tan2_1, double x, double y, double z) {
    if (!(z > 0.0)) return 0.0;
    const double rho2 = x * x + y * y;
    const double r = tan2_1 * rho2 / (z * z);
    if (!(r > 0.0) || r > 1000.0) return 0.0;  // pole, or e^(1 - r) below the smallest double
    const double b = r * exp(1.0 - r);
    const double rho = sqrt(rho2);
    const double cx = x / rho, cy = y / rho;
    double re = 1.0, im = 0.0;
    for (int m = 0; m < k; ++m) {
        const double t = re * cx - im * cy;
        im = re * cy + im * cx;
        re = t;
    }
    return b * re;
}

// Source charges in tree order: q = zeta A, or (zeta - F_R(x, t)) A with the
// forcing on; x is the particle's (sorted) position.
__global__ __launch_bounds__(256) void k_charges(const i32* __restrict__ perm, i64 n,
                                                  const double* __restrict__ zeta,
                                                  const double* __restrict__ area, const double* __restrict__ sx,
                                                  const double* __restrict__ sy, const double* __restrict__ sz,
                                                  ForcingDev f, double* __restrict__ q,
                                                  u32* __restrict__ flags) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const i32 j = perm[i];
    double z = zeta[j];
    if (f.on) {
        const double t = f.t_dev ? *f.t_dev + f.t_base : f.t_base;
        const double a = forcing_ramp(t, f.t_ramp, f.t_total);
        if (a != 0.0) z -= f.amp * a * forcing_shape(f.k, f.tan2_1, sx[i], sy[i], sz[i]);
    }
    const double qi = z * area[j];
    if (!isfinite(qi)) atomicOr(&flags[F_NONFINITE_CHARGE], 1u);  // reported at synchronisation
    q[i] = qi;
}

// F_R(x_i, t) at caller positions (row-major (n, 3)), input order.
__global__ __launch_bounds__(256) void k_forcing_field(i64 n, const double* __restrict__ x, ForcingDev f,
                                                        double* __restrict__ out) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a = forcing_ramp(f.t_base, f.t_ramp, f.t_total);
    out[i] = a == 0.0 ? 0.0 : f.amp * a * forcing_shape(f.k, f.tan2_1, x[3 * i], x[3 * i + 1], x[3 * i + 2]);
}

__global__ void k_forcing_clock(double* t, double value, int set) {
    if (threadIdx.x == 0 && blockIdx.x == 0) t[0] = set ? value : t[0] + value;
}

// ---------------------------------------------------------------------------
// Upward pass (Sec. 3, particle-cluster interaction).  For every node P with
// more than N_T particles:
//   omega_k = sum over the particles y of P of B_k(b(y)) q(y),  b = M_P^{-1} y,
//   w_m     = |b_m1 v1 + b_m2 v2 + b_m3 v3|^d * sum_k (V_ref^{-1})_{km} omega_k
// (w = V^{-T} omega with the node's Vandermonde matrix V = diag(s^d) V_ref),
// B_k = c_k b1^i b2^j b3^(d-i-j) with k running over i, then j.
//
// Every node's weights come straight from its own particles, so no level
// waits for another.  The tree build cut each big node's particle range into
// items of at most UP_CHUNK particles (k_node_counts).  k_upward_items: one
// wave per item, lane l taking particles l, l + 64, ...; the terms
// q b1^i b2^j b3^(d-i-j) of all (i, j) accumulate in registers, then the wave
// adds them across lanes by recursive halving and writes the item's sums.
// k_upward_finish: a workgroup per batch of UP_BATCH big nodes adds each
// node's item sums in item order (deterministic), multiplies the batch by
// V_ref^{-1} as one small matrix product through LDS, and writes the proxy
// points and charges into the nodes' storage slots.
// ---------------------------------------------------------------------------

// index of term (i, j) in the k order
__host__ __device__ constexpr int term_index(int d, int i, int j) { return i * (d + 1) - i * (i - 1) / 2 + j; }

// Recursive halving over the 64 lanes: v holds N partial sums of terms
// [start, start + len) (slots past len are zero).  Lanes with bit MASK set
// keep the upper half and send the lower; partners (lanes differing only in
// that bit) describe the same terms, so each keeps the sum of both.
template <int N, int MASK>
struct WaveHalve {
    __device__ __forceinline__ static void run(const double (&v)[N], int lane, int start, int len,
                                               double* __restrict__ out) {
        constexpr int H = (N + 1) / 2;
        const bool up = (lane & MASK) != 0;
        double nv[H];
#pragma unroll
        for (int t = 0; t < H; ++t) {
            const double lo = v[t];
            const double hi = (t + H < N) ? v[t + H] : 0.0;
            const double send = up ? lo : hi;
            const double keep = up ? hi : lo;
            nv[t] = keep + __shfl_xor(send, MASK, 64);
        }
        if (up) {
            start += H;
            len = len > H ? len - H : 0;
        } else {
            len = len < H ? len : H;
        }
        WaveHalve<H, MASK / 2>::run(nv, lane, start, len, out);
    }
};
template <int N>
struct WaveHalve<N, 0> {
    __device__ __forceinline__ static void run(const double (&v)[N], int, int start, int len,
                                               double* __restrict__ out) {
#pragma unroll
        for (int t = 0; t < N; ++t)
            if (t < len) out[start + t] = v[t];
    }
};

// Terms with I0 <= i <= I1 of one item's particles [lo, hi), summed over the
// wave and written to out[k] (k the term index).
template <int D, int I0, int I1>
__device__ __forceinline__ void item_terms(const double* __restrict__ sx, const double* __restrict__ sy,
                                           const double* __restrict__ sz, const double* __restrict__ q, int lo,
                                           int hi, const NodeGeo& g, double* __restrict__ out) {
    constexpr int M0 = term_index(D, I0, 0), M1 = term_index(D, I1 + 1, 0);
    constexpr int NT = M1 - M0;
    const int lane = threadIdx.x & 63;
    double acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = 0.0;
    const double m00 = g.minv[0][0], m01 = g.minv[0][1], m02 = g.minv[0][2];
    const double m10 = g.minv[1][0], m11 = g.minv[1][1], m12 = g.minv[1][2];
    const double m20 = g.minv[2][0], m21 = g.minv[2][1], m22 = g.minv[2][2];
    // the next particle is loaded while the current one's terms accumulate
    int j = lo + lane;
    double n0 = 0.0, n1 = 0.0, n2 = 0.0, nq = 0.0;
    if (j < hi) n0 = sx[j], n1 = sy[j], n2 = sz[j], nq = q[j];
    for (; j < hi; j += 64) {
        const double y0 = n0, y1 = n1, y2 = n2, qq = nq;
        if (j + 64 < hi) n0 = sx[j + 64], n1 = sy[j + 64], n2 = sz[j + 64], nq = q[j + 64];
        const double b0 = (m00 * y0 + m01 * y1) + m02 * y2;
        const double b1 = (m10 * y0 + m11 * y1) + m12 * y2;
        const double b2 = (m20 * y0 + m21 * y1) + m22 * y2;
        double p1[D + 1], p2[D + 1];
        p1[0] = 1.0;
        p2[0] = 1.0;
#pragma unroll
        for (int t = 1; t <= D; ++t) {
            p1[t] = p1[t - 1] * b1;
            p2[t] = p2[t - 1] * b2;
        }
        double qi = qq;
#pragma unroll
        for (int i = 0; i < I0; ++i) qi *= b0;
#pragma unroll
        for (int i = I0; i <= I1; ++i) {
#pragma unroll
            for (int jj = 0; jj <= D - i; ++jj)
                acc[term_index(D, i, jj) - M0] = __fma_rn(qi, p1[jj] * p2[D - i - jj], acc[term_index(D, i, jj) - M0]);
            qi *= b0;
        }
    }
    WaveHalve<NT, 32>::run(acc, lane, M0, NT, out);
}

// last i of the first group of terms: at most 66 accumulators per pass
__host__ __device__ constexpr int upward_split(int d) {
    int a = d;
    while (a > 0 && term_index(d, a + 1, 0) > 66) --a;
    return a;
}

template <int D>
__global__ __launch_bounds__(256) void k_upward_items(const u32* __restrict__ flags, u32 items_cap,
                                                       const i32* __restrict__ item_node,
                                                       const i32* __restrict__ item_chunk, u32 node_mask,
                                                       const i32* __restrict__ nbeg, const i32* __restrict__ nend,
                                                       const NodeGeo* __restrict__ geo, const double* __restrict__ sx,
                                                       const double* __restrict__ sy, const double* __restrict__ sz,
                                                       const double* __restrict__ q, double* __restrict__ part) {
    constexpr int NP = (D + 1) * (D + 2) / 2;
    constexpr int A = upward_split(D);
    u32 n_items = flags[F_ITEMS];
    if (n_items > items_cap) n_items = items_cap;
    const u32 waves = gridDim.x * (blockDim.x / 64);
    for (u32 it = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); it < n_items; it += waves) {
        const i32 node = item_node[it];
        const i32 b = nbeg[node], e = nend[node];
        const int lo = b + item_chunk[it] * UP_CHUNK;
        const int hi = (lo + UP_CHUNK) < e ? lo + UP_CHUNK : e;
        const NodeGeo& g = geo[(u32)node & node_mask];
        double* out = part + (size_t)it * NP;
        item_terms<D, 0, A>(sx, sy, sz, q, lo, hi, g, out);
        if constexpr (A < D) item_terms<D, A + 1, D>(sx, sy, sz, q, lo, hi, g, out);
    }
}

// Batch j = big nodes [UP_BATCH j, UP_BATCH (j + 1)) of the level lists taken
// in level order.  om[r][k] = c_k * (sum of node r's item sums), then
// w[r][m] = |P_m|^d sum_k om[r][k] (V_ref^{-1})_{km} with V_ref^{-1} staged in
// LDS when it fits (n_p <= 78), else read from memory.  Small batches keep
// many workgroups in flight: the work per node is small, its chain of
// dependent loads is what takes time.
template <int D>
__global__ __launch_bounds__(256) void k_upward_finish(int L, const u32* __restrict__ flags,
                                                        const i32* __restrict__ big_list, u32 per_level,
                                                        const i32* __restrict__ nbeg, const i32* __restrict__ nend,
                                                        const i32* __restrict__ item_base, u32 node_mask,
                                                        const NodeGeo* __restrict__ geo,
                                                        const double* __restrict__ part, RefDev ref, int NPT, int poff,
                                                        const i32* __restrict__ slot, Prox* __restrict__ prox) {
    constexpr int NP = (D + 1) * (D + 2) / 2;
    constexpr bool LDS_V = NP <= 78;
    constexpr int R = UP_BATCH;
    __shared__ double om[R][NP];
    __shared__ double vl[LDS_V ? NP * NP : 1];
    __shared__ double gv[R][9];  // node vertices
    __shared__ i32 slots[R], items[R], bases[R];
    const int tid = threadIdx.x;
    if constexpr (LDS_V) {
        for (int t = tid; t < NP * NP; t += 256) vl[t] = ref.vinv[t];
    }
    const double* __restrict__ V = LDS_V ? vl : ref.vinv;
    // big nodes at levels <= l: the level counts loaded in parallel, then
    // the prefix (LDS, so that no thread indexes a register array)
    __shared__ u32 lvl_end[kMaxLevels + 1];
    if (tid <= L) lvl_end[tid] = flags[F_LEVEL + tid] < per_level ? flags[F_LEVEL + tid] : per_level;
    __syncthreads();
    if (tid == 0)
        for (int l = 1; l <= L; ++l) lvl_end[l] += lvl_end[l - 1];
    __syncthreads();
    const u32 total = lvl_end[L];
    const u32 n_batch = (total + R - 1) / R;
    for (u32 bj = blockIdx.x; bj < n_batch; bj += gridDim.x) {
        const u32 g0 = bj * R;
        const int nr = (total - g0) < (u32)R ? (int)(total - g0) : R;
        if (tid < nr) {
            const u32 gidx = g0 + tid;
            int lvl = 0;
            while (gidx >= lvl_end[lvl]) ++lvl;
            const u32 bi = gidx - (lvl > 0 ? lvl_end[lvl - 1] : 0u);
            const i32 node = big_list[(size_t)lvl * per_level + bi];
            const i32 sl = slot[node];
            slots[tid] = sl;
            items[tid] = (nend[node] - nbeg[node] + UP_CHUNK - 1) / UP_CHUNK;
            bases[tid] = item_base[sl];
            const NodeGeo& g = geo[(u32)node & node_mask];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) gv[tid][3 * a + c] = g.v[a][c];
        }
        __syncthreads();
        for (int o = tid; o < nr * NP; o += 256) {
            const int r = o / NP, k = o - r * NP;
            const size_t base = (size_t)bases[r];
            double sum = 0.0;
            for (int t = 0; t < items[r]; ++t) sum += part[(base + t) * NP + k];
            om[r][k] = ref.coef[k] * sum;
        }
        __syncthreads();
        for (int o = tid; o < nr * NP; o += 256) {
            const int r = o / NP, m = o - r * NP;
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
            int k = 0;
#pragma unroll 4
            for (; k + 4 <= NP; k += 4) {
                a0 = __fma_rn(om[r][k], V[k * NP + m], a0);
                a1 = __fma_rn(om[r][k + 1], V[(k + 1) * NP + m], a1);
                a2 = __fma_rn(om[r][k + 2], V[(k + 2) * NP + m], a2);
                a3 = __fma_rn(om[r][k + 3], V[(k + 3) * NP + m], a3);
            }
            for (; k < NP; ++k) a0 = __fma_rn(om[r][k], V[k * NP + m], a0);
            // proxy point: normalise(b1 v1 + b2 v2 + b3 v3), |.| for the scale
            const double* b = ref.points + 3 * m;
            double p[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) p[c] = (b[0] * gv[r][c] + b[1] * gv[r][3 + c]) + b[2] * gv[r][6 + c];
            const double nrm = sqrt((p[0] * p[0] + p[1] * p[1]) + p[2] * p[2]);
            const double inv = 1.0 / nrm;
            Prox pr;
            pr.x = p[0] * inv;
            pr.y = p[1] * inv;
            pr.z = p[2] * inv;
            pr.w = ipow(nrm, D) * ((a0 + a1) + (a2 + a3));
            prox[(size_t)slots[r] * NPT + poff + m] = pr;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Lower-degree proxy charges from the degree-10 ones (learned form).  The
// degree-d interpolant's space lies inside the degree-10 one, so the degree-d
// charges are the degree-10 point charges re-interpolated:
//   w_d,m = |P_d,m|^d sum_n T_nm w_10,n / |P_10,n|^d,
// P = b_1 v_1 + b_2 v_2 + b_3 v_3 the unnormalised point of reference
// barycentrics b, and T_nm = sum_k (V_ref,d^{-1})_km B_k(b_10,n) a fixed
// reference matrix (the multinomial-scaled basis is homogeneous of degree d,
// so the node's geometry enters only through |P|), stored [n][m] so that the
// lanes (one output m each) read consecutive entries.  The table sits in
// LDS, read once per workgroup (every node reading its 46 KB from L2 cost
// more than the arithmetic); one wave per node, each wave walking its own
// nodes, all levels' nodes in one index space.
// ---------------------------------------------------------------------------
constexpr int kDsWaves = 8;
constexpr int kDsTable = 66 * 88;  // degree 10 -> degrees 4, 6, 8: 66 inputs x 88 outputs
__global__ __launch_bounds__(64 * kDsWaves) void k_downsample(int L, int NB, const u32* __restrict__ flags,
                                                              const i32* __restrict__ big_list, u32 per_level,
                                                              const NodeGeo* __restrict__ geo,
                                                              const i32* __restrict__ slot,
                                                              const double* __restrict__ ref_points,
                                                              const double* __restrict__ T, ClassTab cls, int NPT,
                                                              Prox* __restrict__ prox) {
    __shared__ double Ts[kDsTable];
    __shared__ double src[kDsWaves][3][kMaxNp];
    __shared__ u32 lvl_end[kMaxLevels + 1];  // big nodes at levels <= l
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const u32 lm = (1u << NB) - 1u;
    const int np10 = cls.np[3], poff10 = cls.poff[3];
    const int nout = cls.poff[3];  // points of classes 0..2
    for (int i = threadIdx.x; i < np10 * nout; i += 64 * kDsWaves) Ts[i] = T[i];
    if (threadIdx.x == 0) {
        u32 total = 0;
        for (int lvl = 0; lvl <= L; ++lvl) {
            total += flags[F_LEVEL + lvl] < per_level ? flags[F_LEVEL + lvl] : per_level;
            lvl_end[lvl] = total;
        }
    }
    __syncthreads();
    const u32 total = lvl_end[L];
    // each wave its own nodes; a wave's LDS rows are its own, so it waits
    // only on itself
    for (u32 bi = blockIdx.x * kDsWaves + w; bi < total; bi += gridDim.x * kDsWaves) {
        int lvl = 0;
        while (bi >= lvl_end[lvl]) ++lvl;
        const i64 node = big_list[(size_t)lvl * per_level + (bi - (lvl > 0 ? lvl_end[lvl - 1] : 0u))];
        const NodeGeo& g = geo[node & lm];
        const size_t rec = (size_t)slot[node] * NPT;
        for (int n = lane; n < np10; n += 64) {
            double y[3];
            const double nrm = proxy_point(g, ref_points + 3 * (poff10 + n), y);
            const double w10 = prox[rec + poff10 + n].w;
            for (int c = 0; c < 3; ++c) src[w][c][n] = w10 / ipow(nrm, cls.deg[c]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int o = lane; o < nout; o += 64) {
            const int c = o < cls.poff[1] ? 0 : (o < cls.poff[2] ? 1 : 2);
            double acc = 0.0;
            for (int n = 0; n < np10; ++n) acc += Ts[n * nout + o] * src[w][c][n];
            double y[3];
            const double nrm = proxy_point(g, ref_points + 3 * o, y);
            Prox pr;
            pr.x = y[0];
            pr.y = y[1];
            pr.z = y[2];
            pr.w = ipow(nrm, cls.deg[c]) * acc;
            prox[rec + o] = pr;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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
// the 400 root pairs of every member (never pairs of two members)
__global__ __launch_bounds__(256) void k_trav_init(int members, int NB, const i32* __restrict__ ncnt,
                                                    u64* __restrict__ front, u32 cap, u32* __restrict__ counters) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = g / 400, i = g % 400;
    const u32 t = ((u32)m << NB) + (u32)(i / 20), s = ((u32)m << NB) + (u32)(i % 20);
    const bool ok = m < members && ncnt[t] > 0 && ncnt[s] > 0;
    const u32 slot = wave_append(&counters[C_FRONT], ok);
    if (ok) {
        if (slot < cap) front[slot] = ((u64)t << 32) | (u64)s;
        else atomicOr(&counters[C_OVERFLOW], 1u);
    }
}

__device__ __forceinline__ bool mac_separated(const NodeMac& a, const NodeMac& b, double theta2) {
#pragma clang fp contract(off)
    const double s = a.r + b.r;
    const double dx = a.cx - b.cx;
    const double dy = a.cy - b.cy;
    const double dz = a.cz - b.cz;
    const double R2 = (dx * dx + dy * dy) + dz * dz;
    return s * s < theta2 * R2;
}

// exclusive prefix of v over the 256 threads of the block, *total = sum
__device__ __forceinline__ u32 block_scan_u32(u32 v, u32* wsum, u32* total) {
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

// One round of a traversal level over frontier pairs [r0, r0 + 256 IPT):
// pair r0 + 256 k + tid for k < IPT.  Several pairs per thread keep more
// loads in flight (large frontiers); one pair per thread shortens each
// thread's chain of dependent loads (small frontiers).
template <bool CAND, int IPT>
__device__ __forceinline__ void trav_round(u64 r0, u32 nin, int iter, int fbase, const u64* __restrict__ fin,
                                           u64* __restrict__ fout, u32 cap, const i32* __restrict__ ncnt,
                                           const NodeMac* __restrict__ mac, const i64* __restrict__ level_off_tab,
                                           int L, u32 lm, double theta2, int n_crit, int W, int DB, int dcf,
                                           u64* __restrict__ tlist, u64* __restrict__ nlist,
                                           u64* __restrict__ cand_buf, u32* __restrict__ counters,
                                           u32 (*wsum)[4], u32* bases) {
    const int tid = threadIdx.x;
    u64 keyv[IPT];
    int kind[IPT];
    bool split_t[IPT];
    int nkids[IPT];
    u32 kids[IPT][4];
    u32 tt[IPT], ss[IPT];
    u32 ct = 0, cn = 0, ck = 0, cc = 0;
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const u64 i = r0 + (u64)k * 256 + tid;
        kind[k] = -1;
        split_t[k] = false;
        nkids[k] = 0;
        tt[k] = ss[k] = 0;
        keyv[k] = 0;
        if (i < nin) {
            const u64 pr = fin[i];
            const u32 t = (u32)(pr >> 32), s = (u32)(pr & 0xffffffffu);
            tt[k] = t;
            ss[k] = s;
            const i32 nt = ncnt[t], ns = ncnt[s];
            const bool big_t = nt > n_crit, big_s = ns > n_crit;
            if (mac_separated(mac[t & lm], mac[s & lm], theta2)) {
                kind[k] = (CAND && (big_t || big_s)) ? 4 : (big_t ? 2 : 0) + (big_s ? 1 : 0);
            } else if (!big_t && !big_s) {
                kind[k] = 0;
            } else {
                const int lt = level_of_offset_table(level_off_tab, L, t & lm);
                const int ls = level_of_offset_table(level_off_tab, L, s & lm);
                const bool int_t = big_t && lt < L, int_s = big_s && ls < L;
                bool st = nt >= ns;
                if (st && !int_t) st = false;
                if (!st && !int_s) {
                    if (int_t) st = true;
                    else kind[k] = 0;
                }
                if (kind[k] < 0) {
                    split_t[k] = st;
                    const u32 x = st ? t : s;
                    const int lx = st ? lt : ls;
                    const i64 child0 = (i64)(x & ~lm) + level_off_tab[lx + 1] + 4 * ((i64)(x & lm) - level_off_tab[lx]);
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const u32 cid = (u32)(child0 + c);
                        if (ncnt[cid] > 0) kids[k][nkids[k]++] = cid;
                    }
                }
            }
            // PP entries carry class 0, far entries the class dcf
            const u64 dc = (kind[k] >= 1 && kind[k] <= 3) ? (u64)dcf : 0u;
            keyv[k] = ((u64)t << (W + 1 + DB)) | (dc << (W + 1)) | ((u64)(kind[k] & 1) << W) | (u64)s;
        }
        ct += (kind[k] == 0 || kind[k] == 1) ? 1u : 0u;
        cn += (kind[k] == 2 || kind[k] == 3) ? 1u : 0u;
        cc += kind[k] == 4 ? 1u : 0u;
        ck += (u32)nkids[k];
    }
    u32 tot_t, tot_n, tot_k, tot_c = 0;
    u32 pt = block_scan_u32(ct, wsum[0], &tot_t);
    u32 pn = block_scan_u32(cn, wsum[1], &tot_n);
    u32 pk = block_scan_u32(ck, wsum[2], &tot_k);
    u32 pc = 0;
    if (CAND) pc = block_scan_u32(cc, wsum[3], &tot_c);
    if (tid == 0) {
        bases[0] = tot_t ? atomicAdd(&counters[C_TLIST], tot_t) : 0u;
        bases[1] = tot_n ? atomicAdd(&counters[C_NLIST], tot_n) : 0u;
        bases[2] = tot_k ? atomicAdd(&counters[fbase + iter + 1], tot_k) : 0u;
        bases[3] = tot_c ? atomicAdd(&counters[C_CAND], tot_c) : 0u;
    }
    __syncthreads();
    u32 ot = bases[0] + pt, on = bases[1] + pn, ok = bases[2] + pk, oc = bases[3] + pc;
    bool overflow = false;
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        if (CAND && kind[k] == 4) {
            if (oc < cap) cand_buf[oc] = ((u64)tt[k] << 32) | (u64)ss[k];
            else overflow = true;
            ++oc;
        } else if (kind[k] == 0 || kind[k] == 1) {
            if (ot < cap) tlist[ot] = keyv[k];
            else overflow = true;
            ++ot;
        } else if (kind[k] >= 2) {
            if (on < cap) nlist[on] = keyv[k];
            else overflow = true;
            ++on;
        }
        for (int c = 0; c < nkids[k]; ++c) {
            const u64 pr = split_t[k] ? (((u64)kids[k][c] << 32) | (u64)ss[k]) : (((u64)tt[k] << 32) | (u64)kids[k][c]);
            if (ok < cap) fout[ok] = pr;
            else overflow = true;
            ++ok;
        }
    }
    if (overflow) atomicOr(&counters[C_OVERFLOW], 1u);
    __syncthreads();  // wsum / bases reused by the next round
}

// A frontier that fits one round of the grid at one pair per thread is
// processed that way (measured on the gv_l8 levels: 5-6 us against 13-15 us
// at four per thread); larger ones at TRAV_IPT pairs per thread.
constexpr int TRAV_IPT = 4;

template <bool CAND>
__global__ __launch_bounds__(256) void k_trav_level(
    int iter, int fbase, const u64* __restrict__ fin, u64* __restrict__ fout, u32 cap, const i32* __restrict__ ncnt,
    const NodeMac* __restrict__ mac, const i64* __restrict__ level_off_tab, int L, int NB, double theta2, int n_crit,
    int W, int DB, int dcf, u64* __restrict__ tlist, u64* __restrict__ nlist, u64* __restrict__ cand_buf,
    u32* __restrict__ counters) {
    __shared__ u32 wsum[4][4];
    __shared__ u32 bases[4];
    u32 nin = counters[fbase + iter];
    if (nin > cap) nin = cap;
    const u32 lm = (1u << NB) - 1u;  // local part of a node id
    if ((u64)nin <= (u64)gridDim.x * 256) {
        const u64 r0 = (u64)blockIdx.x * 256;
        if (r0 < nin)
            trav_round<CAND, 1>(r0, nin, iter, fbase, fin, fout, cap, ncnt, mac, level_off_tab, L, lm, theta2, n_crit,
                                W, DB, dcf, tlist, nlist, cand_buf, counters, wsum, bases);
        return;
    }
    const u64 round = (u64)256 * TRAV_IPT;
    for (u64 r0 = (u64)blockIdx.x * round; r0 < nin; r0 += (u64)gridDim.x * round)
        trav_round<CAND, TRAV_IPT>(r0, nin, iter, fbase, fin, fout, cap, ncnt, mac, level_off_tab, L, lm, theta2,
                                   n_crit, W, DB, dcf, tlist, nlist, cand_buf, counters, wsum, bases);
}

// Per-node particle count, and for every node with more than N_T particles a
// storage slot for its proxy records and target coefficients and an entry in
// its level's list (the upward pass walks those lists).  Slots and list
// positions are handed out in any order; only where a node's data lives
// depends on it.
__global__ __launch_bounds__(256) void k_node_counts(const i32* __restrict__ nbeg, const i32* __restrict__ nend,
                                                      i64 n_nodes, int n_crit, int NB, int L,
                                                      const i64* __restrict__ level_off_tab, i32* __restrict__ ncnt,
                                                      i32* __restrict__ slot, u32 slot_cap, i32* __restrict__ big_list,
                                                      u32 per_level, i32* __restrict__ item_node,
                                                      i32* __restrict__ item_chunk, i32* __restrict__ item_base,
                                                      u32 items_cap, u32* __restrict__ flags) {
    const u64 stride = (u64)gridDim.x * blockDim.x;
    const int lane = threadIdx.x & 63;
    for (u64 b0 = (u64)blockIdx.x * blockDim.x; b0 < (u64)n_nodes; b0 += stride) {
        const u64 i = b0 + threadIdx.x;
        const bool ok = i < (u64)n_nodes;
        const i32 c = ok ? nend[i] - nbeg[i] : 0;
        const bool big = ok && c > n_crit;
        const u32 sl = wave_append(&flags[F_SLOT_CTR], big);  // every lane of the wave takes part
        if (big && sl >= slot_cap) atomicOr(&flags[F_SLOTS], 1u);
        if (ok) {
            ncnt[i] = c;
            slot[i] = big ? (i32)(sl < slot_cap ? sl : slot_cap - 1) : -1;
        }
        // level lists: the lanes of a wave at the level of its first big node
        // share one atomic (node ids run level by level, so that is nearly all)
        const int lvl = big ? level_of_offset_table(level_off_tab, L, (i64)(i & (((u64)1 << NB) - 1))) : -1;
        const u64 bm = __ballot(big);
        if (bm) {
            const int l0 = __shfl(lvl, __ffsll((unsigned long long)bm) - 1, 64);
            const bool same = big && lvl == l0;
            u32 pos = wave_append(&flags[F_LEVEL + l0], same);
            if (big && !same) pos = atomicAdd(&flags[F_LEVEL + lvl], 1u);
            if (big) {
                if (pos < per_level) big_list[(size_t)lvl * per_level + pos] = (i32)i;
                else atomicOr(&flags[F_SLOTS], 1u);
            }
        }
        // upward-pass items: ceil(c / UP_CHUNK) per big node, a wave's items
        // reserved with one atomic (exclusive scan over the lanes)
        const u32 ni = big ? (u32)((c + UP_CHUNK - 1) / UP_CHUNK) : 0u;
        u32 incl = ni;
        for (int o = 1; o < 64; o <<= 1) {
            const u32 t = __shfl_up(incl, o, 64);
            if (lane >= o) incl += t;
        }
        const u32 tot = __shfl(incl, 63, 64);
        u32 ib = 0;
        if (lane == 0 && tot > 0) ib = atomicAdd(&flags[F_ITEMS], tot);
        ib = __shfl(ib, 0, 64) + (incl - ni);
        if (big) {
            if (sl < slot_cap && (u64)ib + ni <= (u64)items_cap) {
                item_base[sl] = (i32)ib;
                for (u32 t = 0; t < ni; ++t) {
                    item_node[ib + t] = (i32)i;
                    item_chunk[ib + t] = (i32)t;
                }
            } else {
                atomicOr(&flags[F_SLOTS], 1u);
            }
        }
    }
}

// Segments of sorted lists: entries with the same key >> shift (the target
// node) occupy [seg_beg[.], seg_end[.]).  Arrays
// must be zeroed before.  grid.y = list.
__global__ __launch_bounds__(256) void k_segments(SegLists sg, u32 cap) {
    const int y = blockIdx.y;
    const u64* __restrict__ list = sg.list[y];
    u32 n = *sg.d_n[y];
    if (n > cap) n = cap;
    const int shift = sg.shift[y];
    i32* __restrict__ seg_beg = sg.beg[y];
    i32* __restrict__ seg_end = sg.end[y];
    const u64 stride = (u64)gridDim.x * blockDim.x;
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const u64 t = list[i] >> shift;
        if (i == 0 || (list[i - 1] >> shift) != t) seg_beg[t] = (i32)i;
        if (i + 1 == n || (list[i + 1] >> shift) != t) seg_end[t] = (i32)(i + 1);
    }
}

__global__ __launch_bounds__(256) void k_fill_u32(u32* __restrict__ p, i64 n, u32 v) {
    const u64 stride = (u64)gridDim.x * blockDim.x;
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < (u64)n; i += stride) p[i] = v;
}

// up to kFillMax arrays zeroed in one launch (grid.y = array)
__global__ __launch_bounds__(256) void k_fill_multi(FillSet f) {
    const int y = blockIdx.y;
    u32* __restrict__ p = f.p[y];
    const u64 n = (u64)f.n[y];
    const u64 stride = (u64)gridDim.x * blockDim.x;
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0u;
}

__global__ __launch_bounds__(256) void k_fill_f64(double* __restrict__ p, i64 n, double v) {
    const u64 stride = (u64)gridDim.x * blockDim.x;
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < (u64)n; i += stride) p[i] = v;
}

// Kernel-evaluation count implied by the lists (introspection only).
__global__ __launch_bounds__(256) void k_count_evals(const u64* __restrict__ list, const u32* __restrict__ d_n,
                                                      u32 cap, int W, int DB, ClassTab cls, const i32* __restrict__ nbeg,
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
        const u64 t = k >> (W + 1 + DB), s = k & mask;
        const int ty = (int)((k >> W) & 1);
        const int c = (int)((k >> (W + 1)) & ((1u << DB) - 1u));
        const int np = STC_PICK4(cls.np, c);
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

void launch_bin(hipStream_t s, const double* x, i64 n, const NodeGeo* geo, int L, const MemberOffsets& mo,
                u64* keys, u32* queue, u32* flags) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_bin, dim3(blocks_for(n, 256)), dim3(256), 0, s, x, n, geo, L, mo, keys, queue, flags);
    hipLaunchKernelGGL(k_bin_exact, dim3(64), dim3(256), 0, s, x, geo, L, mo, queue, flags, keys);
}

void launch_gather(hipStream_t s, const u64* keys, i64 n, const double* x, i32* perm, u32* leaf, double* sx,
                   double* sy, double* sz) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather, dim3(blocks_for(n, 256)), dim3(256), 0, s, keys, n, x, perm, leaf, sx, sy, sz);
}

void launch_node_ranges(hipStream_t s, const u32* leaf, i64 n, int L, int NB, i32* nbeg, i32* nend) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_node_ranges, dim3(blocks_for(n, 256)), dim3(256), 0, s, leaf, n, L, NB, nbeg, nend);
}

void launch_charges(hipStream_t s, const i32* perm, i64 n, const double* zeta, const double* area,
                    const double* sx, const double* sy, const double* sz, ForcingDev f, double* q, u32* flags) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_charges, dim3(blocks_for(n, 256)), dim3(256), 0, s, perm, n, zeta, area, sx, sy, sz, f, q,
                       flags);
}

void launch_forcing_field(hipStream_t s, i64 n, const double* x, ForcingDev f, double* out) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_forcing_field, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, x, f, out);
}

void launch_forcing_clock(hipStream_t s, double* t, double value, int set) {
    hipLaunchKernelGGL(k_forcing_clock, dim3(1), dim3(64), 0, s, t, value, set);
}

void launch_upward(hipStream_t s, int L, int NB, const u32* flags, const i32* big_list, u32 per_level,
                   const i32* nbeg, const i32* nend, const i32* item_node, const i32* item_chunk,
                   const i32* item_base, u32 items_cap, const NodeGeo* geo, const double* sx, const double* sy,
                   const double* sz, const double* q, double* part, RefDev ref, int NPT, int poff, const i32* slot,
                   Prox* prox) {
    const u32 mask = (1u << NB) - 1u;
    // items: a persistent grid of 4 waves per workgroup walks the item list;
    // then batches of big nodes (a fixed grid walks them)
    const dim3 gi(1024), bi(256);
    const unsigned gf = (unsigned)std::min<u64>(((u64)(L + 1) * per_level + UP_BATCH - 1) / UP_BATCH, 2048u);
    switch (ref.degree) {
#define STC_UP_CASE(D)                                                                                          \
    case D:                                                                                                     \
        hipLaunchKernelGGL(k_upward_items<D>, gi, bi, 0, s, flags, items_cap, item_node, item_chunk, mask, nbeg, \
                           nend, geo, sx, sy, sz, q, part);                                                      \
        hipLaunchKernelGGL(k_upward_finish<D>, dim3(gf), bi, 0, s, L, flags, big_list, per_level, nbeg, nend,    \
                           item_base, mask, geo, part, ref, NPT, poff, slot, prox);                              \
        break;
        STC_UP_CASE(1) STC_UP_CASE(2) STC_UP_CASE(3) STC_UP_CASE(4) STC_UP_CASE(5) STC_UP_CASE(6) STC_UP_CASE(7)
        STC_UP_CASE(8) STC_UP_CASE(9) STC_UP_CASE(10) STC_UP_CASE(11) STC_UP_CASE(12) STC_UP_CASE(13)
        STC_UP_CASE(14)
#undef STC_UP_CASE
        default: break;
    }
}

void launch_downsample(hipStream_t s, int L, int NB, const u32* flags, const i32* big_list, u32 per_level,
                       const NodeGeo* geo, const i32* slot, const double* ref_points, const double* T, ClassTab cls,
                       int NPT, Prox* prox, int cus) {
    // the learned form's classes are degrees 4, 6, 8 and 10 (stc_create), so
    // the table is 66 x 88; 69 KB of LDS: two workgroups per CU
    const u32 want = std::max<u32>((per_level + kDsWaves - 1) / kDsWaves, 1u);
    const unsigned grid = (unsigned)std::min<u32>(want, (u32)(2 * std::max(cus, 1)));
    hipLaunchKernelGGL(k_downsample, dim3(grid), dim3(64 * kDsWaves), 0, s, L, NB, flags, big_list, per_level, geo,
                       slot, ref_points, T, cls, NPT, prox);
}

void launch_fill_u32(hipStream_t s, u32* p, i64 n, u32 v) {
    if (n <= 0) return;
    const i64 b = blocks_for(n, 256);
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)(b < 4096 ? b : 4096)), dim3(256), 0, s, p, n, v);
}

void launch_fill_zero(hipStream_t s, const FillSet& f) {
    if (f.k <= 0) return;
    i64 mx = 0;
    for (int y = 0; y < f.k; ++y) mx = f.n[y] > mx ? f.n[y] : mx;
    if (mx <= 0) return;
    const i64 b = blocks_for(mx, 256);
    hipLaunchKernelGGL(k_fill_multi, dim3((unsigned)(b < 2048 ? b : 2048), (unsigned)f.k), dim3(256), 0, s, f);
}

void launch_fill_f64(hipStream_t s, double* p, i64 n, double v) {
    if (n <= 0) return;
    const i64 b = blocks_for(n, 256);
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)(b < 4096 ? b : 4096)), dim3(256), 0, s, p, n, v);
}

void launch_node_counts(hipStream_t s, const i32* nbeg, const i32* nend, i64 n_nodes, int n_crit, int NB, int L,
                        const i64* level_off_dev, i32* ncnt, i32* slot, u32 slot_cap, i32* big_list, u32 per_level,
                        i32* item_node, i32* item_chunk, i32* item_base, u32 items_cap, u32* flags) {
    const i64 b = blocks_for(n_nodes, 256);
    hipLaunchKernelGGL(k_node_counts, dim3((unsigned)(b < 2048 ? b : 2048)), dim3(256), 0, s, nbeg, nend, n_nodes,
                       n_crit, NB, L, level_off_dev, ncnt, slot, slot_cap, big_list, per_level, item_node,
                       item_chunk, item_base, items_cap, flags);
}

void launch_traverse_init(hipStream_t s, const TravArgs& t, bool zero_counters) {
    if (zero_counters) launch_fill_u32(s, t.counters, C_COUNT, 0u);
    hipLaunchKernelGGL(k_trav_init, dim3(blocks_for((i64)t.members * 400, 256)), dim3(256), 0, s, t.members, t.NB,
                       t.ncnt, t.front0, t.cap, t.counters);
}

void launch_traverse_levels(hipStream_t s, const TravArgs& t, int fbase, bool cand, u64* cand_buf) {
    const double theta2 = t.theta * t.theta;
    const int iters = 2 * t.L + 2;
    for (int it = 0; it < iters; ++it) {
        const u64* fin = (it % 2 == 0) ? t.front0 : t.front1;
        u64* fout = (it % 2 == 0) ? t.front1 : t.front0;
        if (cand)
            hipLaunchKernelGGL(k_trav_level<true>, dim3(1024), dim3(256), 0, s, it, fbase, fin, fout, t.cap, t.ncnt,
                               t.mac, t.level_off_tab, t.L, t.NB, theta2, t.n_crit, t.W, t.DB, t.dcf, t.tlist,
                               t.nlist, cand_buf, t.counters);
        else
            hipLaunchKernelGGL(k_trav_level<false>, dim3(1024), dim3(256), 0, s, it, fbase, fin, fout, t.cap, t.ncnt,
                               t.mac, t.level_off_tab, t.L, t.NB, theta2, t.n_crit, t.W, t.DB, t.dcf, t.tlist,
                               t.nlist, cand_buf, t.counters);
    }
}

void launch_segments(hipStream_t s, const SegLists& sg, u32 cap) {
    hipLaunchKernelGGL(k_segments, dim3(1024, (unsigned)sg.k), dim3(256), 0, s, sg, cap);
}

void launch_count_evals(hipStream_t s, const u64* list, const u32* d_n, u32 cap, int W, int DB, ClassTab cls,
                        const i32* nbeg, const i32* nend, int target_is_proxy, unsigned long long* out) {
    hipLaunchKernelGGL(k_count_evals, dim3(256), dim3(256), 0, s, list, d_n, cap, W, DB, cls, nbeg, nend,
                       target_is_proxy, out);
}

}  // namespace stc
