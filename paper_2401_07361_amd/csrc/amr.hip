// Adaptive refinement of the particle triangulation (Appendix A; the
// Gaussian-vortex test of Sec. 4.3), on the GPU.
//
// The particles are the vertices of a triangulation whose every initial
// triangle is the root of a refinement tree of depth at most D.  Every
// triangle and every particle that refinement can ever create has a fixed
// slot, numbered on the host once (stc_amr_create): the triangles of root r
// occupy slots r TS .. r TS + TS - 1 (TS = (4^(D+1) - 1) / 3, depth by
// depth, the children of local slot l at depth d at 4 l + c of depth d + 1),
// the particles are the n0 initial ones, then every edge midpoint of the
// depth-D refinement in order of first appearance (a midpoint is one slot
// for the two triangles of its edge).  A pass therefore only flips states:
//
//   crit     C(T) per leaf triangle and per refined triangle whose children
//            are leaves (positions and vorticities at the start of the pass)
//   decide   merge (refined, leaf children, no C) before split (leaf, C,
//            depth < D, its parent not merging); new triangle states
//   mark     live particles = vertices of the new leaves
//   birth    a particle live now but not before: midpoint of its edge's ends,
//            mean absolute vorticity zeta + 2 Omega z of the ends
//   children the four children of a split take the parent's carried area in
//            proportion to their spherical areas (triangles carry their
//            areas: the flow is incompressible; an initial triangle takes
//            its spherical area at the first pass)
//   areas    A_i = sum of carried A_T / 3 over the leaves having i as a
//            vertex, in slot order of the triangles (fixed, repeatable)
//   compact  live particles in slot order into the arrays the tree code
//            reads (x, zeta, A) and the slot of each
//
// The decisions and the new particles follow the same formulas, in the same
// operation order, as the description of the readings in the header (stc.h);
// this file is compiled without floating-point contraction.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "stc.h"

using namespace stc;

namespace {

constexpr u8 T_OFF = 0, T_LEAF = 1, T_REFINED = 2;
constexpr u8 D_NONE = 0, D_MERGE = 1, D_SPLIT = 2;
constexpr int kMaxAmrDepth = 6;

// slots of one root's subtree: depth d starts at (4^d - 1) / 3
__host__ __device__ __forceinline__ int depth_of(int local) {
    int d = 0;
    int start = 1;
    while (local >= start) {
        local -= start;
        start *= 4;
        ++d;
    }
    return d;
}

__host__ __device__ __forceinline__ int depth_start(int d) { return ((1 << (2 * d)) - 1) / 3; }

struct AmrDev {
    i64 ntri, npart;
    int D, TS;
    const i32* tv;      // [ntri][3] particle slots of each triangle slot
    const i32* ends;    // [npart][2] edge ends of a midpoint slot (-1 for initial particles)
    const i32* adj_beg; // [npart + 1] CSR of triangle slots having the particle as a vertex
    const i32* adj;
    u8 *state, *state_new, *crit, *dec;
    double* tarea;      // [ntri] carried area (negative: not yet set)
    u8 *alive, *alive_new;
    double *x, *z;      // slot state: positions (npart x 3), vorticity
    double* area_slot;
    // compact state
    double *cx, *cz, *ca;
    i32* slot_of;
    u32* counters;      // [0] live particles after the last pass, [1] leaves, [2] merges, [3] splits, [4..] scan
    u32* block_sums;
};

__device__ __forceinline__ double tri_area_dev(const double* a, const double* b, const double* c) {
    const double bxc0 = b[1] * c[2] - b[2] * c[1];
    const double bxc1 = b[2] * c[0] - b[0] * c[2];
    const double bxc2 = b[0] * c[1] - b[1] * c[0];
    const double trip = fabs((a[0] * bxc0 + a[1] * bxc1) + a[2] * bxc2);
    const double ab = (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
    const double bc = (b[0] * c[0] + b[1] * c[1]) + b[2] * c[2];
    const double ca = (c[0] * a[0] + c[1] * a[1]) + c[2] * a[2];
    return 2.0 * atan2(trip, ((1.0 + ab) + bc) + ca);
}

__device__ __forceinline__ bool children_all_leaves(const u8* st, i64 s, int local, int d, int TS) {
    const i64 root = s - local;
    const int cl = depth_start(d + 1) + 4 * (local - depth_start(d));
    for (int c = 0; c < 4; ++c)
        if (st[root + cl + c] != T_LEAF) return false;
    return true;
}

__global__ __launch_bounds__(256) void k_amr_crit(AmrDev a, double eps1, double eps2) {
    const i64 s = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.ntri) return;
    const int local = (int)(s % a.TS);
    const int d = depth_of(local);
    const u8 st = a.state[s];
    u8 c = 0;
    if (st == T_LEAF || (st == T_REFINED && d < a.D && children_all_leaves(a.state, s, local, d, a.TS))) {
        const i32 i = a.tv[3 * s], j = a.tv[3 * s + 1], k = a.tv[3 * s + 2];
        double area = a.tarea[s];
        if (area < 0.0) {  // an initial triangle at the first pass
            area = tri_area_dev(a.x + 3 * (i64)i, a.x + 3 * (i64)j, a.x + 3 * (i64)k);
            a.tarea[s] = area;
        }
        const double zi = a.z[i], zj = a.z[j], zk = a.z[k];
        const double circ = area * (((zi + zj) + zk) / 3.0);
        const double zmax = fmax(fmax(zi, zj), zk), zmin = fmin(fmin(zi, zj), zk);
        c = (fabs(circ) >= eps1 || (zmax - zmin) >= eps2) ? 1 : 0;
    }
    a.crit[s] = c;
}

// merge / split decision of slot s (see the file comment)
__device__ __forceinline__ bool merges(const AmrDev& a, i64 s, int local, int d) {
    return a.state[s] == T_REFINED && d < a.D && children_all_leaves(a.state, s, local, d, a.TS) && !a.crit[s];
}

__global__ __launch_bounds__(256) void k_amr_decide(AmrDev a) {
    const i64 s = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.ntri) return;
    const int local = (int)(s % a.TS);
    const int d = depth_of(local);
    u8 dec = D_NONE;
    if (merges(a, s, local, d)) {
        dec = D_MERGE;
    } else if (a.state[s] == T_LEAF && a.crit[s] && d < a.D) {
        bool parent_merges = false;
        if (d > 0) {
            const int pl = depth_start(d - 1) + (local - depth_start(d)) / 4;
            parent_merges = merges(a, s - local + pl, pl, d - 1);
        }
        if (!parent_merges) dec = D_SPLIT;
    }
    a.dec[s] = dec;
}

__global__ __launch_bounds__(256) void k_amr_apply(AmrDev a) {
    const i64 s = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.ntri) return;
    const int local = (int)(s % a.TS);
    const int d = depth_of(local);
    u8 st = a.state[s];
    const u8 dec = a.dec[s];
    if (dec == D_MERGE) st = T_LEAF;
    else if (dec == D_SPLIT) st = T_REFINED;
    else if (d > 0) {
        const int pl = depth_start(d - 1) + (local - depth_start(d)) / 4;
        const u8 pd = a.dec[s - local + pl];
        if (pd == D_MERGE) st = T_OFF;
        else if (pd == D_SPLIT) st = T_LEAF;
    }
    a.state_new[s] = st;
}

__global__ __launch_bounds__(256) void k_amr_clear_alive(AmrDev a) {
    const i64 v = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < a.npart) a.alive_new[v] = 0;
}

__global__ __launch_bounds__(256) void k_amr_mark(AmrDev a) {
    const i64 s = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.ntri || a.state_new[s] != T_LEAF) return;
    a.alive_new[a.tv[3 * s]] = 1;
    a.alive_new[a.tv[3 * s + 1]] = 1;
    a.alive_new[a.tv[3 * s + 2]] = 1;
}

__global__ __launch_bounds__(256) void k_amr_birth(AmrDev a, double omega) {
    const i64 v = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= a.npart || !a.alive_new[v] || a.alive[v]) return;
    const i32 ia = a.ends[2 * v], ib = a.ends[2 * v + 1];
    if (ia < 0 || ib < 0) return;  // an initial particle has no edge (and is never born)
    const double* xa = a.x + 3 * (i64)ia;
    const double* xb = a.x + 3 * (i64)ib;
    const double s0 = xa[0] + xb[0], s1 = xa[1] + xb[1], s2 = xa[2] + xb[2];
    const double r = sqrt((s0 * s0 + s1 * s1) + s2 * s2);
    const double m0 = s0 / r, m1 = s1 / r, m2 = s2 / r;
    const double two_om = 2.0 * omega;
    const double absv = 0.5 * ((a.z[ia] + two_om * xa[2]) + (a.z[ib] + two_om * xb[2]));
    a.x[3 * v] = m0;
    a.x[3 * v + 1] = m1;
    a.x[3 * v + 2] = m2;
    a.z[v] = absv - two_om * m2;
}

// carried areas of the children of every split (after the births: the
// children's vertices have positions)
__global__ __launch_bounds__(256) void k_amr_child_areas(AmrDev a) {
    const i64 s = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.ntri || a.dec[s] != D_SPLIT) return;
    const int local = (int)(s % a.TS);
    const int d = depth_of(local);
    const i64 c0 = s - local + depth_start(d + 1) + 4 * (local - depth_start(d));
    double g[4];
    for (int c = 0; c < 4; ++c) {
        const i64 t = c0 + c;
        const i32 i = a.tv[3 * t], j = a.tv[3 * t + 1], k = a.tv[3 * t + 2];
        g[c] = tri_area_dev(a.x + 3 * (i64)i, a.x + 3 * (i64)j, a.x + 3 * (i64)k);
    }
    const double gs = ((g[0] + g[1]) + g[2]) + g[3];
    const double A = a.tarea[s];
    for (int c = 0; c < 4; ++c) a.tarea[c0 + c] = A * (g[c] / gs);
}

// per particle: its weight from the carried areas of its leaves, then the
// new live flags become current
__global__ __launch_bounds__(256) void k_amr_areas(AmrDev a) {
    const i64 v = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= a.npart) return;
    double acc = 0.0;
    if (a.alive_new[v]) {
        for (i32 e = a.adj_beg[v]; e < a.adj_beg[v + 1]; ++e) {
            const i32 t = a.adj[e];
            if (a.state_new[t] != T_LEAF) continue;
            acc += a.tarea[t] / 3.0;
        }
    }
    a.area_slot[v] = acc;
}

__global__ __launch_bounds__(256) void k_amr_commit(AmrDev a) {
    const i64 s = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < a.ntri) a.state[s] = a.state_new[s];
    if (s < a.npart) a.alive[s] = a.alive_new[s];
}

// compaction of the live particles in slot order: per-block counts, a scan
// of the block counts in one workgroup, then each block writes its part
__global__ __launch_bounds__(256) void k_amr_count(AmrDev a) {
    __shared__ u32 wsum[4];
    const i64 v = (i64)blockIdx.x * 256 + threadIdx.x;
    const u32 f = (v < a.npart && a.alive[v]) ? 1u : 0u;
    const u64 bal = __ballot(f);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = (u32)__popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) a.block_sums[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

__global__ __launch_bounds__(256) void k_amr_scan_blocks(AmrDev a, u32 nblocks) {
    __shared__ u32 part[256];
    // each thread sums a contiguous run of blocks, then an exclusive scan of
    // the 256 run totals, then each run is rewritten as exclusive offsets
    const u32 per = (nblocks + 255) / 256;
    const u32 b0 = threadIdx.x * per, b1 = min(b0 + per, nblocks);
    u32 sum = 0;
    for (u32 b = b0; b < b1; ++b) sum += a.block_sums[b];
    part[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        u32 run = 0;
        for (int k = 0; k < 256; ++k) {
            const u32 t = part[k];
            part[k] = run;
            run += t;
        }
        a.counters[0] = run;
    }
    __syncthreads();
    u32 off = part[threadIdx.x];
    for (u32 b = b0; b < b1; ++b) {
        const u32 t = a.block_sums[b];
        a.block_sums[b] = off;
        off += t;
    }
}

__global__ __launch_bounds__(256) void k_amr_compact(AmrDev a) {
    __shared__ u32 wsum[4];
    const i64 v = (i64)blockIdx.x * 256 + threadIdx.x;
    const bool f = v < a.npart && a.alive[v];
    const u64 bal = __ballot(f);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) wsum[w] = (u32)__popcll(bal);
    __syncthreads();
    if (!f) return;
    u32 base = a.block_sums[blockIdx.x];
    for (int k = 0; k < w; ++k) base += wsum[k];
    const u32 o = base + (u32)__popcll(bal & ((1ull << lane) - 1ull));
    a.cx[3 * (i64)o] = a.x[3 * v];
    a.cx[3 * (i64)o + 1] = a.x[3 * v + 1];
    a.cx[3 * (i64)o + 2] = a.x[3 * v + 2];
    a.cz[o] = a.z[v];
    a.ca[o] = a.area_slot[v];
    a.slot_of[o] = (i32)v;
}

// the compact state (after time steps) back into the slots
__global__ __launch_bounds__(256) void k_amr_scatter(AmrDev a, i64 n, const double* __restrict__ x,
                                                    const double* __restrict__ z) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const i64 v = a.slot_of[i];
    a.x[3 * v] = x[3 * i];
    a.x[3 * v + 1] = x[3 * i + 1];
    a.x[3 * v + 2] = x[3 * i + 2];
    a.z[v] = z[i];
}

// per-pass statistics: live leaves, merges and splits
__global__ __launch_bounds__(256) void k_amr_stats(AmrDev a) {
    const i64 s = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.ntri) return;
    if (a.state[s] == T_LEAF) atomicAdd(&a.counters[1], 1u);
    if (a.dec[s] == D_MERGE) atomicAdd(&a.counters[2], 1u);
    if (a.dec[s] == D_SPLIT) atomicAdd(&a.counters[3], 1u);
}

unsigned blocks(i64 n) { return (unsigned)std::max<i64>(1, (n + 255) / 256); }

// host tables of the fixed slot numbering
struct AmrTables {
    std::vector<i32> tv, ends, adj_beg, adj;
    i64 ntri = 0, npart = 0;
    int TS = 0;
};

bool build_tables(i64 n0, i64 nf, const int32_t* faces, int D, AmrTables& t) {
    t.TS = depth_start(D + 1);
    t.ntri = nf * (i64)t.TS;
    t.tv.assign((size_t)t.ntri * 3, -1);
    t.ends.assign((size_t)n0 * 2, -1);
    std::unordered_map<u64, i32> mid;
    mid.reserve((size_t)(3 * nf * t.TS / 2 + 16));
    i64 np = n0;
    auto midpoint = [&](i32 a, i32 b) -> i32 {
        const u64 key = ((u64)(u32)std::min(a, b) << 32) | (u32)std::max(a, b);
        auto it = mid.find(key);
        if (it != mid.end()) return it->second;
        const i32 id = (i32)np++;
        mid.emplace(key, id);
        t.ends.push_back(a);
        t.ends.push_back(b);
        return id;
    };
    for (i64 r = 0; r < nf; ++r) {
        const i64 base = r * t.TS;
        for (int k = 0; k < 3; ++k) {
            const i32 v = faces[3 * r + k];
            if (v < 0 || v >= n0) return false;
            t.tv[3 * base + k] = v;
        }
        for (int d = 0; d < D; ++d) {
            const int s0 = depth_start(d), s1 = depth_start(d + 1);
            for (int l = s0; l < s1; ++l) {
                const i32* p = &t.tv[3 * (base + l)];
                const i32 a = p[0], b = p[1], c = p[2];
                const i32 mab = midpoint(a, b), mbc = midpoint(b, c), mca = midpoint(c, a);
                const i32 ch[4][3] = {{a, mab, mca}, {mab, b, mbc}, {mca, mbc, c}, {mab, mbc, mca}};
                const int cl = s1 + 4 * (l - s0);
                for (int q = 0; q < 4; ++q)
                    for (int k = 0; k < 3; ++k) t.tv[3 * (base + cl + q) + k] = ch[q][k];
            }
        }
        if (np >= 0x7fffffffLL) return false;
    }
    t.npart = np;
    // CSR: triangle slots of each particle, in increasing slot order
    std::vector<i32> cnt((size_t)np + 1, 0);
    for (i64 s = 0; s < t.ntri; ++s)
        for (int k = 0; k < 3; ++k) ++cnt[(size_t)t.tv[3 * s + k] + 1];
    for (i64 v = 0; v < np; ++v) cnt[(size_t)v + 1] += cnt[(size_t)v];
    t.adj_beg = cnt;
    t.adj.assign((size_t)cnt[(size_t)np], 0);
    std::vector<i32> fill(cnt.begin(), cnt.end() - 1);
    for (i64 s = 0; s < t.ntri; ++s)
        for (int k = 0; k < 3; ++k) t.adj[(size_t)fill[(size_t)t.tv[3 * s + k]]++] = (i32)s;
    return true;
}

constexpr size_t kAlign = 256;

struct Carve {
    char* base = nullptr;
    size_t off = 0;
    template <typename T>
    void take(T** p, size_t count) {
        if (count == 0) count = 1;
        off = (off + kAlign - 1) & ~(kAlign - 1);
        if (base) *p = reinterpret_cast<T*>(base + off);
        off += count * sizeof(T);
    }
};

}  // namespace

struct stc_amr {
    stc_amr_params p{};
    hipStream_t stream = nullptr;
    AmrTables tab;
    i64 n0 = 0, nf = 0;
    i64 n = 0;  // live particles (host copy, after stc_amr_particles)
    i32 *tv = nullptr, *ends = nullptr, *adj_beg = nullptr, *adj = nullptr;
    u8 *state = nullptr, *state_new = nullptr, *crit = nullptr, *dec = nullptr, *alive = nullptr,
       *alive_new = nullptr;
    double* tarea = nullptr;
    double *x = nullptr, *z = nullptr, *area_slot = nullptr, *cx = nullptr, *cz = nullptr, *ca = nullptr;
    i32* slot_of = nullptr;
    u32 *counters = nullptr, *block_sums = nullptr;
    std::string err;

    AmrDev dev() const {
        AmrDev a{};
        a.ntri = tab.ntri;
        a.npart = tab.npart;
        a.D = p.max_levels;
        a.TS = tab.TS;
        a.tv = tv;
        a.ends = ends;
        a.adj_beg = adj_beg;
        a.adj = adj;
        a.state = state;
        a.state_new = state_new;
        a.crit = crit;
        a.dec = dec;
        a.tarea = tarea;
        a.alive = alive;
        a.alive_new = alive_new;
        a.x = x;
        a.z = z;
        a.area_slot = area_slot;
        a.cx = cx;
        a.cz = cz;
        a.ca = ca;
        a.slot_of = slot_of;
        a.counters = counters;
        a.block_sums = block_sums;
        return a;
    }
};

namespace {

void carve_amr(stc_amr* m, Carve& cv) {
    const size_t nt = (size_t)m->tab.ntri, np = (size_t)m->tab.npart;
    cv.take(&m->tv, 3 * nt);
    cv.take(&m->ends, 2 * np);
    cv.take(&m->adj_beg, np + 1);
    cv.take(&m->adj, m->tab.adj.size());
    cv.take(&m->state, nt);
    cv.take(&m->state_new, nt);
    cv.take(&m->crit, nt);
    cv.take(&m->dec, nt);
    cv.take(&m->tarea, nt);
    cv.take(&m->alive, np);
    cv.take(&m->alive_new, np);
    cv.take(&m->x, 3 * np);
    cv.take(&m->z, np);
    cv.take(&m->area_slot, np);
    cv.take(&m->cx, 3 * np);
    cv.take(&m->cz, np);
    cv.take(&m->ca, np);
    cv.take(&m->slot_of, np);
    cv.take(&m->counters, 8);
    cv.take(&m->block_sums, (np + 255) / 256);
}

stc_status plan_amr(stc_amr* m, const stc_amr_params* p, int64_t n0, int64_t n_faces, const int32_t* h_faces) {
    if (!p || !h_faces || n0 < 3 || n_faces < 1 || n0 >= 0x7fffffffLL) return STC_ERR_INVALID_ARG;
    if (p->max_levels < 0 || p->max_levels > kMaxAmrDepth || !(p->eps1 >= 0.0) || !(p->eps2 >= 0.0) ||
        !std::isfinite(p->omega))
        return STC_ERR_INVALID_ARG;
    m->p = *p;
    m->n0 = n0;
    m->nf = n_faces;
    try {
        if (!build_tables(n0, n_faces, h_faces, p->max_levels, m->tab)) return STC_ERR_INVALID_ARG;
    } catch (...) {
        return STC_ERR_ALLOC;
    }
    return STC_OK;
}

// one adaptation pass on the slot state (enqueued on m->stream)
void enqueue_pass(stc_amr* m) {
    hipStream_t s = m->stream;
    const AmrDev a = m->dev();
    hipLaunchKernelGGL(k_amr_crit, dim3(blocks(a.ntri)), dim3(256), 0, s, a, m->p.eps1, m->p.eps2);
    hipLaunchKernelGGL(k_amr_decide, dim3(blocks(a.ntri)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_amr_apply, dim3(blocks(a.ntri)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_amr_clear_alive, dim3(blocks(a.npart)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_amr_mark, dim3(blocks(a.ntri)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_amr_birth, dim3(blocks(a.npart)), dim3(256), 0, s, a, m->p.omega);
    hipLaunchKernelGGL(k_amr_child_areas, dim3(blocks(a.ntri)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_amr_areas, dim3(blocks(a.npart)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_amr_commit, dim3(blocks(std::max(a.ntri, a.npart))), dim3(256), 0, s, a);
}

// compaction of the live particles (and pass statistics)
void enqueue_compact(stc_amr* m) {
    hipStream_t s = m->stream;
    const AmrDev a = m->dev();
    const unsigned nb = blocks(a.npart);
    launch_fill_u32(s, m->counters + 1, 3, 0u);
    hipLaunchKernelGGL(k_amr_stats, dim3(blocks(a.ntri)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_amr_count, dim3(nb), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_amr_scan_blocks, dim3(1), dim3(256), 0, s, a, nb);
    hipLaunchKernelGGL(k_amr_compact, dim3(nb), dim3(256), 0, s, a);
}

stc_status fail(stc_amr* m, stc_status st, const char* msg) {
    if (m) m->err = msg;
    return st;
}

bool aligned8(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

}  // namespace

extern "C" {

stc_status stc_amr_workspace_size(const stc_amr_params* p, int64_t n0, int64_t n_faces, const int32_t* h_faces,
                                  size_t* bytes, int64_t* max_particles) {
    if (!bytes) return STC_ERR_INVALID_ARG;
    *bytes = 0;
    stc_amr* m = new (std::nothrow) stc_amr();
    if (!m) return STC_ERR_ALLOC;
    stc_status st = plan_amr(m, p, n0, n_faces, h_faces);
    if (st == STC_OK) {
        Carve cv;
        carve_amr(m, cv);
        *bytes = cv.off;
        if (max_particles) *max_particles = m->tab.npart;
    }
    delete m;
    return st;
}

stc_status stc_amr_create(const stc_amr_params* p, int64_t n0, int64_t n_faces, const int32_t* h_faces, void* d_ws,
                          size_t ws_bytes, void* hip_stream, stc_amr** out) {
    if (!out) return STC_ERR_INVALID_ARG;
    *out = nullptr;
    stc_amr* m = new (std::nothrow) stc_amr();
    if (!m) return STC_ERR_ALLOC;
    stc_status st = plan_amr(m, p, n0, n_faces, h_faces);
    if (st != STC_OK) {
        delete m;
        return st;
    }
    Carve cv;
    carve_amr(m, cv);
    if (!d_ws || (reinterpret_cast<uintptr_t>(d_ws) & (kAlign - 1)) || ws_bytes < cv.off) {
        delete m;
        return STC_ERR_WORKSPACE;
    }
    cv = Carve{static_cast<char*>(d_ws), 0};
    carve_amr(m, cv);
    m->stream = static_cast<hipStream_t>(hip_stream);
    hipStream_t s = m->stream;
    const AmrTables& t = m->tab;
    // initial state: every root a leaf, the other slots off, the initial particles live
    std::vector<u8> st0((size_t)t.ntri, T_OFF);
    for (i64 r = 0; r < m->nf; ++r) st0[(size_t)(r * t.TS)] = T_LEAF;
    const std::vector<double> ta0((size_t)t.ntri, -1.0);
    std::vector<u8> al0((size_t)t.npart, 0);
    std::fill(al0.begin(), al0.begin() + m->n0, (u8)1);
    std::vector<i32> slot0((size_t)m->n0);
    for (i64 v = 0; v < m->n0; ++v) slot0[(size_t)v] = (i32)v;
    auto up = [&](void* dst, const void* src, size_t bytes) {
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) == hipSuccess;
    };
    bool ok = up(m->tv, t.tv.data(), t.tv.size() * sizeof(i32)) && up(m->ends, t.ends.data(), t.ends.size() * sizeof(i32)) &&
              up(m->adj_beg, t.adj_beg.data(), t.adj_beg.size() * sizeof(i32)) &&
              up(m->adj, t.adj.data(), t.adj.size() * sizeof(i32)) && up(m->state, st0.data(), st0.size()) &&
              up(m->tarea, ta0.data(), ta0.size() * sizeof(double)) &&
              up(m->alive, al0.data(), al0.size()) && up(m->slot_of, slot0.data(), slot0.size() * sizeof(i32));
    launch_fill_u32(s, m->counters, 8, 0u);
    if (!ok || hipStreamSynchronize(s) != hipSuccess) {
        delete m;
        return STC_ERR_DEVICE;
    }
    m->n = m->n0;
    *out = m;
    return STC_OK;
}

stc_status stc_amr_destroy(stc_amr* m) {
    if (!m) return STC_ERR_INVALID_ARG;
    (void)hipStreamSynchronize(m->stream);
    delete m;
    return STC_OK;
}

stc_status stc_amr_set_state(stc_amr* m, int64_t n, const double* d_x, const double* d_zeta) {
    if (!m) return STC_ERR_INVALID_ARG;
    if (n != m->n) return fail(m, STC_ERR_INVALID_ARG, "n must be the current particle count");
    if (n > 0 && (!d_x || !d_zeta || !aligned8(d_x) || !aligned8(d_zeta)))
        return fail(m, STC_ERR_INVALID_ARG, "NULL or misaligned pointer");
    if (n == 0) return STC_OK;
    const AmrDev a = m->dev();
    hipLaunchKernelGGL(k_amr_scatter, dim3(blocks(n)), dim3(256), 0, m->stream, a, (i64)n, d_x, d_zeta);
    return hipGetLastError() == hipSuccess ? STC_OK : fail(m, STC_ERR_DEVICE, "scatter failed");
}

stc_status stc_amr_adapt(stc_amr* m) {
    if (!m) return STC_ERR_INVALID_ARG;
    enqueue_pass(m);
    enqueue_compact(m);
    if (hipGetLastError() != hipSuccess) return fail(m, STC_ERR_DEVICE, "adaptation pass failed");
    u32 h[4];
    if (hipMemcpyAsync(h, m->counters, sizeof(h), hipMemcpyDeviceToHost, m->stream) != hipSuccess ||
        hipStreamSynchronize(m->stream) != hipSuccess)
        return fail(m, STC_ERR_DEVICE, "reading the particle count failed");
    m->n = h[0];
    return STC_OK;
}

stc_status stc_amr_particles(stc_amr* m, int64_t* n, double** d_x, double** d_zeta, double** d_area) {
    if (!m) return STC_ERR_INVALID_ARG;
    if (n) *n = m->n;
    if (d_x) *d_x = m->cx;
    if (d_zeta) *d_zeta = m->cz;
    if (d_area) *d_area = m->ca;
    return STC_OK;
}

stc_status stc_amr_stats(stc_amr* m, int64_t* n_particles, int64_t* n_leaves, int64_t* merged, int64_t* split,
                         int64_t* max_particles) {
    if (!m) return STC_ERR_INVALID_ARG;
    u32 h[4];
    if (hipMemcpyAsync(h, m->counters, sizeof(h), hipMemcpyDeviceToHost, m->stream) != hipSuccess ||
        hipStreamSynchronize(m->stream) != hipSuccess)
        return fail(m, STC_ERR_DEVICE, "reading counters failed");
    if (n_particles) *n_particles = m->n;
    if (n_leaves) *n_leaves = h[1];
    if (merged) *merged = h[2];
    if (split) *split = h[3];
    if (max_particles) *max_particles = m->tab.npart;
    return STC_OK;
}

stc_status stc_amr_copy_slots(stc_amr* m, int64_t cap, int32_t* h_slots, int32_t* h_ends) {
    if (!m || cap < 0) return STC_ERR_INVALID_ARG;
    if (hipStreamSynchronize(m->stream) != hipSuccess) return fail(m, STC_ERR_DEVICE, "synchronisation failed");
    const i64 k = std::min<i64>(cap, m->n);
    if (h_slots && k > 0 && hipMemcpy(h_slots, m->slot_of, k * sizeof(i32), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(m, STC_ERR_DEVICE, "copy failed");
    if (h_ends) {
        const i64 e = std::min<i64>(cap, m->tab.npart);
        std::memcpy(h_ends, m->tab.ends.data(), (size_t)(2 * e) * sizeof(i32));
    }
    return STC_OK;
}

const char* stc_amr_last_error(const stc_amr* m) { return m ? m->err.c_str() : ""; }

}  // extern "C"

namespace stc {
hipStream_t amr_stream(const stc_amr* m) { return m->stream; }
}  // namespace stc
