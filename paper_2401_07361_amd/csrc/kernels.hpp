// Host launchers of the HIP kernels (internal to the library).
#pragma once

#include "common.hpp"

struct stc_amr;

namespace stc {

// Degree classes: a context evaluates far-field interactions at one degree
// (class 0) or, with learned gating, at the degree class each list entry
// carries (degrees 4, 6, 8, 10).  Per class: points per node, offset of the
// class's points inside a node's record of NPT points, degree, offset of its
// np x np matrices in the concatenated reference tables.
struct ClassTab {
    int np[4], poff[4], deg[4], qoff[4];
};

#define STC_PICK4(arr, c) ((c) == 0 ? (arr)[0] : (c) == 1 ? (arr)[1] : (c) == 2 ? (arr)[2] : (arr)[3])

// List keys: (t << (W + 1 + DB)) | (class << (W + 1)) | (type << W) | s, with
// DB = 0 (single degree) or 2 (degree classes).  The target-particle list is
// grouped by t, the target-proxy list by (t, class).

// k_tree.hip
void launch_bin(hipStream_t s, const double* x, i64 n, const NodeGeo* geo, int L, const MemberOffsets& mo,
                u64* keys, u32* queue, u32* flags);
void launch_gather(hipStream_t s, const u64* keys, i64 n, const double* x, i32* perm, u32* leaf,
                   double* sx, double* sy, double* sz);
void launch_node_ranges(hipStream_t s, const u32* leaf, i64 n, int L, int NB, i32* nbeg, i32* nend);
// Vorticity forcing of the polar-vortex collapse experiment (Sec. 4.4): the
// charges become q = (zeta - F_R(x, t)) A with
// F_R = amp A(t) B(lat) cos(k lon), amp = (3/5) Omega k^2.  The time is
// t_base, or *t_dev + t_base when t_dev is set (RK4 stages under a graph).
struct ForcingDev {
    int on, k;
    double amp, tan2_1, t_ramp, t_total, t_base;
    const double* t_dev;
};
// q = zeta A in tree order (forced: (zeta - F_R) A); a non-finite charge
// raises flags[F_NONFINITE_CHARGE]
void launch_charges(hipStream_t s, const i32* perm, i64 n, const double* zeta, const double* area,
                    const double* sx, const double* sy, const double* sz, ForcingDev f, double* q, u32* flags);
// F_R(x_i, f.t_base) at n positions in input order
void launch_forcing_field(hipStream_t s, i64 n, const double* x, ForcingDev f, double* out);
// single-thread update of the forcing clock: *t = set ? value : *t + value
void launch_forcing_clock(hipStream_t s, double* t, double value, int set);
void launch_upward(hipStream_t s, int L, int NB, const u32* flags, const i32* big_list, u32 per_level,
                   const i32* nbeg, const i32* nend, const i32* item_node, const i32* item_chunk,
                   const i32* item_base, u32 items_cap, const NodeGeo* geo, const double* sx, const double* sy,
                   const double* sz, const double* q, double* part, RefDev ref, int NPT, int poff, const i32* slot,
                   Prox* prox);
void launch_downsample(hipStream_t s, int L, int NB, const u32* flags, const i32* big_list, u32 per_level,
                       const NodeGeo* geo, const i32* slot, const double* ref_points, const double* T, ClassTab cls,
                       int NPT, Prox* prox, int cus);
void launch_node_counts(hipStream_t s, const i32* nbeg, const i32* nend, i64 n_nodes, int n_crit, int NB, int L,
                        const i64* level_off_dev, i32* ncnt, i32* slot, u32 slot_cap, i32* big_list, u32 per_level,
                        i32* item_node, i32* item_chunk, i32* item_base, u32 items_cap, u32* flags);
// Traversal: the root pairs of every member into front0 (counters zeroed),
// then 2L + 2 level iterations from front0 whose frontier lengths live at
// counters[fbase + k].  Far entries get degree class dcf; with `cand`, pairs
// that are separated and have a side with more than n_crit particles go to
// cand_buf (counter C_CAND) instead of the lists.
struct TravArgs {
    int members, NB, L, n_crit, W, DB, dcf;
    double theta;
    const i32* ncnt;
    const NodeMac* mac;
    const i64* level_off_tab;
    u64 *front0, *front1;
    u32 cap;
    u64 *tlist, *nlist;
    u32* counters;
};
void launch_traverse_init(hipStream_t s, const TravArgs& t, bool zero_counters = true);
void launch_traverse_levels(hipStream_t s, const TravArgs& t, int fbase, bool cand, u64* cand_buf);
// segments of up to two sorted lists in one launch
struct SegLists {
    const u64* list[2];
    const u32* d_n[2];
    int shift[2];
    i32* beg[2];
    i32* end[2];
    int k;
};
void launch_segments(hipStream_t s, const SegLists& sg, u32 cap);
void launch_fill_u32(hipStream_t s, u32* p, i64 n, u32 v);
// zero up to kFillMax u32 arrays in one launch
constexpr int kFillMax = 6;
struct FillSet {
    u32* p[kFillMax];
    i64 n[kFillMax];
    int k;
    void add(void* ptr, i64 count) {
        p[k] = static_cast<u32*>(ptr);
        n[k] = count;
        ++k;
    }
};
void launch_fill_zero(hipStream_t s, const FillSet& f);
void launch_fill_f64(hipStream_t s, double* p, i64 n, double v);
void launch_count_evals(hipStream_t s, const u64* list, const u32* d_n, u32 cap, int W, int DB, ClassTab cls,
                        const i32* nbeg, const i32* nend, int target_is_proxy, unsigned long long* out);

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
    const u32* level_big;  // per level: number of nodes with more than N_T particles
    const i32* perm;
    i64 n;
    RefDev ref;          // all classes' tables concatenated (class offsets in cls)
    ClassTab cls;
    int ndeg;            // degree classes in use (1 or 4)
    int DB;              // class bits in the list keys (0 or 2)
    int NPT;             // points per node record (sum over classes)
    int precision;
    int denominator;
    u32 node_mask;       // local part of a node id
    int NB, LB;          // node id bits per member, leaf key bits per member
    // launch shapes of the persistent segment kernels
    int near_threads, near_grid, far_threads, far_grid;
    int stream;          // 1: the stream function's logarithmic kernel, output psi (n values)
    // learned form: class c's Lagrange basis at the degree-10 reference
    // points, [(poff_c + m) * np10 + n], and c_k (V_ref,10^{-1})_kn, [n * np10 + k]
    const double* up_T;
    const double* up_H;
    // nodes with more than N_T particles, per level (k_far_finish), and the
    // learned form's degree classes present at each target node (by slot)
    const i32* big_list;
    u32 per_level;
    int cus;  // compute units of the device (workgroups of the one-per-CU finish kernels)
    u32* cls_mask;
};

void launch_near(hipStream_t s, const EvalArgs& a, u32 type_mask);
void launch_far_targets(hipStream_t s, const EvalArgs& a);
void launch_far_finish(hipStream_t s, const EvalArgs& a);
void launch_l2p_finalize(hipStream_t s, const EvalArgs& a, bool do_far, double* d_u, bool accumulate);
int direct_blocks_per_cu(int precision, int denominator);
int direct_targets_per_block(int precision);
void direct_split(i64 n, i64 m, int cus, int blocks_per_cu, int targets_per_block, u32* chunks, i64* chunk_len);
void launch_direct(hipStream_t s, i64 n, const double* x, const double* zeta, const double* area, i64 m,
                   const i64* targets, int precision, int denominator, u32 chunks, i64 chunk_len, double* part,
                   double* u, int stream);

// k_mlp.hip -- the learned form's network (12 -> 64 -> 64 -> 4, BF16 on the matrix cores)
int mlp_param_count();
i64 mlp_workspace_floats(i64 n_batch);
void launch_mlp_forward(hipStream_t s, const u16* X, i64 n, const u32* d_n, u32 cap, const u16* P, float* out);
int launch_mlp_grad(hipStream_t s, const u16* X, const float* Y, const i32* idx, i64 nb, const u16* P, float* ws);
void launch_mlp_reduce_adam(hipStream_t s, const float* ws, int nwaves, float* grad, float* loss, float* master,
                            float* m1, float* m2, u16* P, float lr, float beta1, float beta2, float eps, int step);
void launch_mlp_batch_index(hipStream_t s, i64 n, i64 base, i64 nb, u64 a, u64 c, i32* idx);
void launch_mlp_round(hipStream_t s, const float* master, u16* P);
// the bias-shift grid of the calibration: 0, then 200 values geometric in [1e-3, 64]
struct CalibGrid {
    static constexpr int K = 201;
    double d[K];
};
// device workspace bytes of launch_mlp_calibrate for n samples
i64 calib_workspace_bytes(i64 n);
// output-bias calibration (all on the device): Q = P with b3[0] -= da and
// b3[1..3] += dc, shifts = {da, dc}
void launch_mlp_calibrate(hipStream_t s, const u16* X, const float* Y, i64 n, const u16* P, double max_false_accept,
                          double max_under_class, void* ws, u16* Q, double* shifts);
// 4 pi sqrt(mean |u_i|^2) over n velocities (n, 3), to *out (one workgroup,
// fixed summation order)
void launch_label_scale(hipStream_t s, const double* u, i64 n, double* out);

// k_learned.hip -- gated traversal of the learned form (single member)
struct LearnedArgs {
    const u64* cand;         // candidate pairs (t << 32 | s), count at counters[C_CAND]
    u32* counters;
    u32 cap;
    const i32* ncnt;
    const i32* nbeg;
    const i32* nend;
    const NodeMac* mac;
    const NodeGeo* geo;
    const i64* level_off_tab;
    int L, n_crit, W, DB;
    const double* qabs;      // per node: sum of |q| and of q over its particles
    const double* qsum;
    const i32* slot;
    const Prox* prox;        // proxy records (class 0 = degree 4 first in each record)
    int NPT;
    u16* feat;               // cap x 16 BF16 features
    float* out;              // cap x 4 network outputs
    const u16* model;        // BF16 parameters
    u64* tlist;
    u64* nlist;
    u64* front;              // frontier of the fallback traversal (counter C_FRONT2)
};
void launch_node_charge_sums(hipStream_t s, const i32* nbeg, const i32* nend, const i64* level_off_host, int L,
                             const double* q, double* qabs, double* qsum);
void launch_features(hipStream_t s, const LearnedArgs& a);
void launch_mlp_forward_list(hipStream_t s, const LearnedArgs& a);
void launch_resolve(hipStream_t s, const LearnedArgs& a, bool use_model);
void launch_pair_errors(hipStream_t s, const LearnedArgs& la, const EvalArgs& a, int dist2, u32 lim, double* err);
void launch_labels(hipStream_t s, const LearnedArgs& la, u32 lim, const double* err, double tol, float* y);

// the stream an adaptive-mesh object enqueues on (amr.hip)
hipStream_t amr_stream(const stc_amr* m);
}  // namespace stc
