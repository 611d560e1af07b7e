// Host launchers of the HIP kernels (internal to the library).
#pragma once

#include "common.hpp"

namespace stc {

// k_tree.hip
void launch_bin(hipStream_t s, const double* x, i64 n, const NodeGeo* geo, int L, const MemberOffsets& mo,
                u64* keys, u32* flags);
void launch_gather(hipStream_t s, const u64* keys, i64 n, const double* x, i32* perm, u32* leaf,
                   double* sx, double* sy, double* sz);
void launch_node_ranges(hipStream_t s, const u32* leaf, i64 n, int L, int NB, i32* nbeg, i32* nend);
void launch_charges(hipStream_t s, const i32* perm, i64 n, const double* zeta, const double* area, double* q);
void launch_upward(hipStream_t s, int members, int NB, const i32* nbeg, const i32* nend, const i64* level_off_host,
                   int L, int n_crit, const NodeGeo* geo, const double* sx, const double* sy, const double* sz,
                   const double* q, RefDev ref, const i32* slot, Prox* prox);
void launch_node_counts(hipStream_t s, const i32* nbeg, const i32* nend, i64 n_nodes, int n_crit, i32* ncnt,
                        i32* slot, u32 slot_cap, u32* flags);
void launch_traverse(hipStream_t s, int members, int NB, const i32* ncnt, const NodeMac* mac,
                     const i64* level_off_tab, int L, double theta, int n_crit, int W, u64* front0, u64* front1,
                     u32 cap, u64* tlist, u64* nlist, u32* counters);
void launch_segments(hipStream_t s, const u64* list, const u32* d_n, u32 cap, int W, i32* seg_beg, i32* seg_end);
void launch_fill_u32(hipStream_t s, u32* p, i64 n, u32 v);
void launch_fill_f64(hipStream_t s, double* p, i64 n, double v);
void launch_count_evals(hipStream_t s, const u64* list, const u32* d_n, u32 cap, int W, int np, const i32* nbeg,
                        const i32* nend, int target_is_proxy, unsigned long long* out);

// k_eval.hip
struct EvalArgs {
    const u64* tlist;
    const u64* nlist;
    const u32* counters;
    u32 cap;
    int W;
    const i32* tseg_end;
    const i32* nseg_beg;
    const i32* nseg_end;
    const i32* nbeg;
    const i32* nend;
    const i32* ncnt;
    int n_crit;
    const NodeGeo* geo;
    const i64* level_off_tab;
    int L;
    const double* sx;
    const double* sy;
    const double* sz;
    const double* sq;
    const i32* slot;     // storage slot of each node with more than N_T particles
    const Prox* prox;    // interpolation points with proxy charges, slots x np
    double* alpha;       // target-side coefficients, slots x np x 3
    double* Wacc;        // per-particle sums, n x 3 (tree order)
    const u32* leaf;
    const i32* perm;
    i64 n;
    RefDev ref;
    int precision;
    int denominator;
    u32 node_mask;       // local part of a node id
    int NB, LB;          // node id bits per member, leaf key bits per member
    // launch shapes of the persistent segment kernels
    int near_threads, near_grid, far_threads, far_grid;
};

void launch_near(hipStream_t s, const EvalArgs& a, u32 type_mask);
void launch_far_targets(hipStream_t s, const EvalArgs& a);
void launch_l2p_finalize(hipStream_t s, const EvalArgs& a, bool do_far, double* d_u, bool accumulate);
void launch_direct(hipStream_t s, i64 n, const double* x, const double* zeta, const double* area, i64 m,
                   const i64* targets, int precision, int denominator, double* u);

}  // namespace stc
