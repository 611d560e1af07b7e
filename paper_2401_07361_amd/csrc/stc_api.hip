// C ABI of the spherical tree code (declared in include/stc.h).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "stc.h"

using namespace stc;

// alignment of the caller's workspace and of every buffer carved from it
constexpr size_t kWorkspaceAlign = 256;

struct stc_ctx {
    stc_params p{};
    int L = 0, np = 0, W = 0;
    // ensembles: node id = (member << NB) | local id, leaf key bits LB = 2L + 5
    int max_members = 1, members = 1, NB = 0, LB = 0;
    i64 n_max = 0, n_max_member = 0;
    i64 n_local = 0;      // nodes of one member's tree
    i64 n_nodes = 0;      // length of the per-node arrays: ((max_members - 1) << NB) + n_local
    i64 used_nodes = 0;   // the part the last build touched
    u32 slot_cap = 0;     // nodes with proxy charges that fit the proxy / coefficient storage
    u32 per_level = 0;    // capacity of each level's list of such nodes
    i32* big_list = nullptr;
    // upward pass: each such node's particles cut into items of UP_CHUNK
    u32 items_cap = 0;
    i32 *item_node = nullptr, *item_chunk = nullptr, *item_base = nullptr;
    double* upart = nullptr;  // items_cap x n_p partial sums
    u32 cap = 0;
    hipStream_t stream = nullptr;
    int cus = 256;
    stc_launch_config shape_default{};
    std::map<int, stc_launch_config> shapes;  // per size class (bits of the particle count)
    std::vector<i64> offsets;                 // member offsets of the last build
    std::vector<NodeGeo> geo_host;
    // degree classes: 1 (the context's degree) or 4 (degrees 4, 6, 8, 10:
    // learned gating); list keys carry DB class bits; a node's proxy record
    // holds NPT points, the classes' points one after the other
    bool learned = false;
    int ndeg = 1, DB = 0, NPT = 0, fb_class = 0;
    ClassTab cls{};
    RefTables ref_host[4];
    u64* cand = nullptr;          // candidate pairs of the gated traversal
    const u64* cand_view = nullptr;  // where the last pass left them (sorted for samples)
    u16* feat = nullptr;          // their features (BF16, 16 per candidate)
    float* mlp_out = nullptr;     // network outputs per candidate
    double *qabs = nullptr, *qsum = nullptr;  // per-node charge sums
    double* ref_T = nullptr;      // degree-10 -> lower-degree re-interpolation, [n][o] (n: degree-10 point)
    double* up_T = nullptr;       // T transposed, [poff_c + m][n]: class c's Lagrange basis at the degree-10 points
    double* up_H = nullptr;       // degree-10 coefficients from values, [n][k] = c_k (V_ref,10^{-1})_kn
    u32* cls_mask = nullptr;      // degree classes with far-field work at each target node (by slot)
    const uint16_t* model = nullptr;  // BF16 network parameters (caller's), or null: reject every candidate
    std::vector<i64> level_off_host;
    // device buffers (all carved from the caller's workspace in stc_create)
    NodeGeo* geo = nullptr;
    NodeMac* mac = nullptr;
    i32* ncnt = nullptr;
    i32* slot = nullptr;
    i64* level_off = nullptr;
    double *ref_points = nullptr, *ref_vinv = nullptr, *ref_vinvT = nullptr, *ref_coef = nullptr;
    int* ref_expo = nullptr;
    u64 *keys_a = nullptr, *keys_b = nullptr, *keys_sorted = nullptr;
    i32* perm = nullptr;
    u32* leaf = nullptr;
    double *sx = nullptr, *sy = nullptr, *sz = nullptr, *sq = nullptr;
    i32 *nbeg = nullptr, *nend = nullptr;
    Prox* prox = nullptr;
    double *alpha = nullptr, *Wacc = nullptr;
    u64 *front0 = nullptr, *front1 = nullptr;
    u64 *tlist_a = nullptr, *tlist_b = nullptr, *nlist_a = nullptr, *nlist_b = nullptr;
    u64 *tlist = nullptr, *nlist = nullptr;
    i32 *tseg_beg = nullptr, *tseg_end = nullptr, *nseg_beg = nullptr, *nseg_end = nullptr;
    u32* counters = nullptr;
    u32* flags = nullptr;
    unsigned long long* evals = nullptr;
    // radix sort scratch (see k_sort.hip)
    u32* sort_zero = nullptr;
    u64* sort_status = nullptr;
    u32* sort_epoch = nullptr;
    int hist_blocks = 0;  // tiles of 4096 keys in the longest array sorted
    // RK4 buffers
    double *rk_x = nullptr, *rk_z = nullptr, *rk_u = nullptr, *rk_xacc = nullptr, *rk_zacc = nullptr;
    // one captured RK4 step, replayed per step (key: the arguments it was captured for)
    hipStream_t cap_stream = nullptr;
    // the upward pass runs here, concurrently with the traversal (they
    // depend only on the tree build); ev_fork / ev_join order it
    hipStream_t side_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // set while the learned form's upward pass runs on side_stream: the
    // gating waits on ev_join before it reads the node charges
    bool gate_waits_upward = false;
    hipGraphExec_t rk_exec = nullptr;
    i64 rk_n = -1;
    std::vector<i64> rk_offsets;
    const void *rk_px = nullptr, *rk_pz = nullptr, *rk_pa = nullptr;
    double rk_dt = 0.0, rk_om = 0.0;
    // vorticity forcing (stc_set_forcing); forcing_t: the device clock RK4 steps read
    bool forcing_on = false;
    stc_forcing forcing{};
    double* forcing_t = nullptr;
    // phase timing: 7 events per recorded evaluation
    std::vector<hipEvent_t> tev;
    int t_max = 0, t_used = 0, t_phase = -1;
    u32 t_mask = 0x3f;  // phases bracketed by events
    // state
    i64 n = -1;
    const double* x = nullptr;
    bool have_tree = false, have_upward = false, have_lists = false;
    void* ws = nullptr;     // the caller's workspace (all device buffers)
    size_t ws_bytes = 0;
    std::string err;
};

static void rk4_drop_graph(stc_ctx* c);

namespace {

const char* kStatusText[] = {"ok", "invalid argument", "interaction list capacity exceeded", "HIP device error",
                             "call out of order", "host allocation failed",
                             "workspace or scratch buffer too small or misaligned",
                             "non-finite particle position, vorticity or area"};

// Phase timing of the evaluation being recorded: an event pair (begin, end)
// per timed phase, recorded on the stream the phase runs on (phases may run
// on two streams at once; each event on a stream costs a few microseconds
// between kernels, so only the timed phases record).  The end of phase 5
// closes the evaluation.
void phase_begin(stc_ctx* c, int p) {
    if (c->t_max == 0 || c->t_used >= c->t_max) return;
    if ((c->t_mask >> p) & 1u) (void)hipEventRecord(c->tev[(size_t)c->t_used * 12 + 2 * p], c->stream);
}

void phase_end(stc_ctx* c, int p) {
    if (c->t_max == 0 || c->t_used >= c->t_max) return;
    if ((c->t_mask >> p) & 1u) (void)hipEventRecord(c->tev[(size_t)c->t_used * 12 + 2 * p + 1], c->stream);
    if (p == 5) ++c->t_used;
}

stc_status fail(stc_ctx* c, stc_status st, const std::string& msg) {
    if (c) c->err = msg;
    return st;
}

stc_status check_launch(stc_ctx* c, const char* where) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, STC_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
    return STC_OK;
}

// Device buffers of a context, carved from the caller's workspace one after
// the other, each at a 256-byte boundary.  With base null only the total
// size is computed (stc_workspace_size).
struct Carver {
    char* base = nullptr;
    size_t off = 0;
    template <typename T>
    void take(T** p, size_t count) {
        if (count == 0) count = 1;
        off = (off + kWorkspaceAlign - 1) & ~(kWorkspaceAlign - 1);
        if (base) *p = reinterpret_cast<T*>(base + off);
        off += count * sizeof(T);
    }
};

bool aligned8(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

SortScratch sort_scratch(const stc_ctx* c) {
    return SortScratch{c->sort_zero, c->sort_status, c->sort_epoch, c->flags + F_SORT_SPIN, c->hist_blocks};
}

int bits_for(i64 v) {
    int b = 0;
    while (((i64)1 << b) < v) ++b;
    return b;
}

int size_class(i64 n) { return bits_for(std::max<i64>(n, 1)); }

stc_launch_config shape_for(const stc_ctx* c, i64 n) {
    auto it = c->shapes.find(size_class(n));
    return it != c->shapes.end() ? it->second : c->shape_default;
}

// workgroups of a persistent segment kernel: a multiple of 8 (one per XCD slot)
int grid_for(const stc_ctx* c, int per_cu) { return std::max(8, ((c->cus * per_cu + 7) / 8) * 8); }

bool valid_shape(const stc_launch_config* s) {
    auto ok_threads = [](int t) { return t == 128 || t == 256 || t == 512; };
    return s && ok_threads(s->near_threads) && ok_threads(s->far_threads) && s->near_blocks_per_cu >= 1 &&
           s->near_blocks_per_cu <= 64 && s->far_blocks_per_cu >= 1 && s->far_blocks_per_cu <= 64;
}

// tables of degree class k
RefDev ref_dev(const stc_ctx* c, int k = 0) {
    RefDev r;
    const int poff = c->cls.poff[k], qoff = c->cls.qoff[k];
    r.points = c->ref_points + 3 * poff;
    r.vinv = c->ref_vinv + qoff;
    r.vinvT = c->ref_vinvT + qoff;
    r.expo = c->ref_expo + 3 * poff;
    r.coef = c->ref_coef + poff;
    r.degree = c->cls.deg[k];
    r.np = c->cls.np[k];
    return r;
}

EvalArgs eval_args(stc_ctx* c) {
    EvalArgs a{};
    a.tlist = c->tlist;
    a.nlist = c->nlist;
    a.counters = c->counters;
    a.cap = c->cap;
    a.W = c->W;
    a.tseg_end = c->tseg_end;
    a.nseg_beg = c->nseg_beg;
    a.nseg_end = c->nseg_end;
    a.nbeg = c->nbeg;
    a.nend = c->nend;
    a.ncnt = c->ncnt;
    a.n_crit = c->p.n_crit;
    a.geo = c->geo;
    a.level_off_tab = c->level_off;
    a.L = c->L;
    a.sx = c->sx;
    a.sy = c->sy;
    a.sz = c->sz;
    a.sq = c->sq;
    a.slot = c->slot;
    a.prox = c->prox;
    a.alpha = c->alpha;
    a.Wacc = c->Wacc;
    a.leaf = c->leaf;
    a.level_big = c->flags + F_LEVEL;
    a.perm = c->perm;
    a.n = c->n;
    a.ref = ref_dev(c, 0);
    a.ref.points = c->ref_points;  // class offsets are applied in the kernels
    a.ref.vinv = c->ref_vinv;
    a.ref.vinvT = c->ref_vinvT;
    a.ref.expo = c->ref_expo;
    a.ref.coef = c->ref_coef;
    a.cls = c->cls;
    a.ndeg = c->ndeg;
    a.DB = c->DB;
    a.NPT = c->NPT;
    a.precision = c->p.precision;
    a.denominator = c->p.denominator;
    a.node_mask = (u32)(((u64)1 << c->NB) - 1);
    a.NB = c->NB;
    a.LB = c->LB;
    const stc_launch_config sh = shape_for(c, c->n);
    a.near_threads = sh.near_threads;
    a.near_grid = grid_for(c, sh.near_blocks_per_cu);
    a.far_threads = sh.far_threads;
    a.far_grid = grid_for(c, sh.far_blocks_per_cu);
    a.up_T = c->up_T;
    a.up_H = c->up_H;
    a.big_list = c->big_list;
    a.per_level = c->per_level;
    a.cus = c->cus;
    a.cls_mask = c->cls_mask;
    return a;
}

stc_status validate_params(const stc_params* p, i64 n_max) {
    if (!p) return STC_ERR_INVALID_ARG;
    if (!(p->theta > 0.0 && p->theta <= 1.0)) return STC_ERR_INVALID_ARG;
    if (p->degree < 1 || p->degree > kMaxDegree) return STC_ERR_INVALID_ARG;
    if (p->n_crit < 1) return STC_ERR_INVALID_ARG;
    if (p->max_level < -1 || p->max_level > 12) return STC_ERR_INVALID_ARG;
    if (p->precision != STC_FP64 && p->precision != STC_FP32) return STC_ERR_INVALID_ARG;
    if (p->denominator != STC_DEN_DOT && p->denominator != STC_DEN_DIST2) return STC_ERR_INVALID_ARG;
    if (p->precision == STC_FP32 && p->denominator != STC_DEN_DIST2) return STC_ERR_INVALID_ARG;
    if (p->list_capacity < 0 || p->list_capacity > 0x7fffffffLL) return STC_ERR_INVALID_ARG;
    if (p->flags & ~(STC_FLAG_EAGER_RK4 | STC_FLAG_LEARNED)) return STC_ERR_INVALID_ARG;
    if (!(p->theta_max >= 0.0 && p->theta_max <= 1.0)) return STC_ERR_INVALID_ARG;
    if (p->flags & STC_FLAG_LEARNED) {
        if (p->degree != 4 && p->degree != 6 && p->degree != 8 && p->degree != 10) return STC_ERR_INVALID_ARG;
        if (p->theta_max > 0.0 && p->theta_max < p->theta) return STC_ERR_INVALID_ARG;
    }
    if (n_max < 0 || n_max >= 0x7fffffffLL) return STC_ERR_INVALID_ARG;
    return STC_OK;
}

// Checks member offsets (host array of members + 1 entries) against the
// context; returns the total particle count or -1.
i64 check_offsets(const stc_ctx* c, int members, const int64_t* h_off) {
    if (members < 1 || members > c->max_members || !h_off || h_off[0] != 0) return -1;
    for (int m = 0; m < members; ++m)
        if (h_off[m + 1] < h_off[m]) return -1;
    const i64 n = h_off[members];
    return n <= c->n_max ? n : -1;
}

// Tree build of `members` particle sets concatenated in d_x (member m owns
// [off[m], off[m+1])).
stc_status do_build(stc_ctx* c, int members, const i64* off, const double* d_x) {
    hipStream_t s = c->stream;
    const i64 n = off[members];
    c->n = n;
    c->x = d_x;
    c->members = members;
    c->offsets.assign(off, off + members + 1);
    c->used_nodes = ((i64)(members - 1) << c->NB) + c->n_local;
    c->have_tree = true;
    c->have_upward = false;
    c->have_lists = false;
    phase_begin(c, 0);
    {
        FillSet f{};
        f.add(c->flags, F_COUNT);
        f.add(c->nbeg, c->used_nodes);
        f.add(c->nend, c->used_nodes);
        f.add(c->sort_zero, kSortZeroWords);
        launch_fill_zero(s, f);
    }
    if (n == 0) {
        launch_fill_u32(s, reinterpret_cast<u32*>(c->ncnt), c->used_nodes, 0u);
        phase_end(c, 0);
        return check_launch(c, "tree_build");
    }
    MemberOffsets mo{};
    mo.m = members;
    for (int m = 0; m <= members; ++m) mo.off[m] = off[m];
    // the sort's second key buffer is free until the sort: it holds the
    // queue of points located exactly
    launch_bin(s, d_x, n, c->geo, c->L, mo, c->keys_a, reinterpret_cast<u32*>(c->keys_b), c->flags);
    radix_sort(s, c->keys_a, c->keys_b, nullptr, (u32)n, 32, 32 + c->LB + bits_for(members),
               sort_scratch(c), &c->keys_sorted);
    launch_gather(s, c->keys_sorted, n, d_x, c->perm, c->leaf, c->sx, c->sy, c->sz);
    launch_node_ranges(s, c->leaf, n, c->L, c->NB, c->nbeg, c->nend);
    launch_node_counts(s, c->nbeg, c->nend, c->used_nodes, c->p.n_crit, c->NB, c->L, c->level_off, c->ncnt, c->slot,
                       c->slot_cap, c->big_list, c->per_level, c->item_node, c->item_chunk, c->item_base,
                       c->items_cap, c->flags);
    phase_end(c, 0);
    return check_launch(c, "tree_build");
}

// Parameter ranges stc_set_forcing and stc_forcing_field accept.
bool forcing_valid(const stc_forcing* f) {
    const double half_pi = 1.5707963267948966;
    return f->k >= 0 && f->k <= 16 && std::isfinite(f->omega) && f->lat1 > 0.0 && f->lat1 < half_pi &&
           f->t_ramp > 0.0 && std::isfinite(f->t_ramp) && f->t_total >= 2.0 * f->t_ramp &&
           std::isfinite(f->t_total) && std::isfinite(f->time);
}

// Device form of a forcing at time t_base (amplitude (3/5) omega k^2).
ForcingDev forcing_dev(const stc_forcing& h, double t_base, const double* t_dev) {
    ForcingDev f{};
    const double tl = tan(h.lat1);
    f.on = 1;
    f.k = h.k;
    f.amp = 0.6 * h.omega * (double)h.k * (double)h.k;
    f.tan2_1 = tl * tl;
    f.t_ramp = h.t_ramp;
    f.t_total = h.t_total;
    f.t_base = t_base;
    f.t_dev = t_dev;
    return f;
}

// Charges (forced at the forcing's host time, or with stage_clock at the
// device clock plus t_off: the RK4 stages, whose start time lives on the
// device so that a captured step can be replayed), then the proxy charges.
stc_status do_upward(stc_ctx* c, const double* d_zeta, const double* d_area, bool stage_clock = false,
                     double t_off = 0.0) {
    hipStream_t s = c->stream;
    phase_begin(c, 1);
    ForcingDev f{};
    if (c->forcing_on)
        f = stage_clock ? forcing_dev(c->forcing, t_off, c->forcing_t) : forcing_dev(c->forcing, c->forcing.time, nullptr);
    launch_charges(s, c->perm, c->n, d_zeta, d_area, c->sx, c->sy, c->sz, f, c->sq, c->flags);
    if (c->n > 0) {
        // the highest class from the particles; the others (learned form) by
        // re-interpolating each node's own record of the highest class
        const int top = c->ndeg - 1;
        launch_upward(s, c->L, c->NB, c->flags, c->big_list, c->per_level, c->nbeg, c->nend, c->item_node,
                      c->item_chunk, c->item_base, c->items_cap, c->geo, c->sx, c->sy, c->sz, c->sq, c->upart,
                      ref_dev(c, top), c->NPT, c->cls.poff[top], c->slot, c->prox);
        if (top > 0)
            launch_downsample(s, c->L, c->NB, c->flags, c->big_list, c->per_level, c->geo, c->slot, c->ref_points,
                              c->ref_T, c->cls, c->NPT, c->prox, c->cus);
    }
    if (c->learned && c->n > 0)
        launch_node_charge_sums(s, c->nbeg, c->nend, c->level_off_host.data(), c->L, c->sq, c->qabs, c->qsum);
    phase_end(c, 1);
    c->have_upward = true;
    return check_launch(c, "upward");
}

LearnedArgs learned_args(stc_ctx* c) {
    LearnedArgs l{};
    l.cand = c->cand;
    l.counters = c->counters;
    l.cap = c->cap;
    l.ncnt = c->ncnt;
    l.nbeg = c->nbeg;
    l.nend = c->nend;
    l.mac = c->mac;
    l.geo = c->geo;
    l.level_off_tab = c->level_off;
    l.L = c->L;
    l.n_crit = c->p.n_crit;
    l.W = c->W;
    l.DB = c->DB;
    l.qabs = c->qabs;
    l.qsum = c->qsum;
    l.slot = c->slot;
    l.prox = c->prox;
    l.NPT = c->NPT;
    l.feat = c->feat;
    l.out = c->mlp_out;
    l.model = c->model;
    l.tlist = c->tlist_a;
    l.nlist = c->nlist_a;
    l.front = c->front0;
    return l;
}

TravArgs trav_args(stc_ctx* c, double theta, int dcf) {
    TravArgs t{};
    t.members = c->members;
    t.NB = c->NB;
    t.L = c->L;
    t.n_crit = c->p.n_crit;
    t.W = c->W;
    t.DB = c->DB;
    t.dcf = dcf;
    t.theta = theta;
    t.ncnt = c->ncnt;
    t.mac = c->mac;
    t.level_off_tab = c->level_off;
    t.front0 = c->front0;
    t.front1 = c->front1;
    t.cap = c->cap;
    t.tlist = c->tlist_a;
    t.nlist = c->nlist_a;
    t.counters = c->counters;
    return t;
}

stc_status do_traverse(stc_ctx* c) {
    hipStream_t s = c->stream;
    phase_begin(c, 2);
    {
        // traversal counters and the segment tables of the sorted lists
        FillSet f{};
        f.add(c->counters, C_COUNT);
        f.add(c->tseg_beg, c->used_nodes);
        f.add(c->tseg_end, c->used_nodes);
        f.add(c->nseg_beg, c->used_nodes << c->DB);
        f.add(c->nseg_end, c->used_nodes << c->DB);
        f.add(c->sort_zero, kSortZeroWords);
        launch_fill_zero(s, f);
    }
    if (!c->learned) {
        const TravArgs t = trav_args(c, c->p.theta, 0);
        launch_traverse_init(s, t, false);
        launch_traverse_levels(s, t, C_FRONT, false, nullptr);
    } else {
        // gated traversal (learned form): pairs separated at theta_max with a
        // side of more than N_T particles are candidates; the network accepts
        // each at a degree class or rejects it; rejected pairs are traversed
        // by the plain method (theta, the fallback degree) from there on
        const TravArgs tc = trav_args(c, c->p.theta_max, 0);
        launch_traverse_init(s, tc, false);
        launch_traverse_levels(s, tc, C_FRONT, true, c->cand);
        LearnedArgs la = learned_args(c);
        c->cand_view = c->cand;
        if (c->gate_waits_upward && hipStreamWaitEvent(s, c->ev_join, 0) != hipSuccess)
            return fail(c, STC_ERR_DEVICE, "stream join failed");
        if (c->model) {
            launch_features(s, la);
            launch_mlp_forward_list(s, la);
        }
        launch_resolve(s, la, c->model != nullptr);
        const TravArgs tf = trav_args(c, c->p.theta, c->fb_class);
        launch_traverse_levels(s, tf, C_FRONT2, false, nullptr);
    }
    const int bits = 2 * c->W + 1 + c->DB;
    const SortScratch sc = sort_scratch(c);
    {
        u64* keys[2] = {c->tlist_a, c->nlist_a};
        u64* tmp[2] = {c->tlist_b, c->nlist_b};
        const u32* cnt[2] = {c->counters + C_TLIST, c->counters + C_NLIST};
        u64* res[2];
        radix_sort_batch(s, 2, keys, tmp, cnt, c->cap, 0, bits, sc, res);
        c->tlist = res[0];
        c->nlist = res[1];
    }
    SegLists sg{{c->tlist, c->nlist},
                {c->counters + C_TLIST, c->counters + C_NLIST},
                {c->W + 1 + c->DB, c->W + 1 + c->DB},
                {c->tseg_beg, c->nseg_beg},
                {c->tseg_end, c->nseg_end},
                2};
    launch_segments(s, sg, c->cap);
    phase_end(c, 2);
    c->have_lists = true;
    return check_launch(c, "traverse");
}

// The context's side stream and its fork / join events, created on first use.
stc_status side_ready(stc_ctx* c) {
    if (!c->side_stream && hipStreamCreateWithFlags(&c->side_stream, hipStreamNonBlocking) != hipSuccess) {
        c->side_stream = nullptr;
        return fail(c, STC_ERR_DEVICE, "creating the side stream failed");
    }
    if (!c->ev_fork && hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess) {
        c->ev_fork = nullptr;
        return fail(c, STC_ERR_DEVICE, "hipEventCreate failed");
    }
    if (!c->ev_join && hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
        c->ev_join = nullptr;
        return fail(c, STC_ERR_DEVICE, "hipEventCreate failed");
    }
    return STC_OK;
}

// The upward pass and the traversal.  Both read only what the tree build
// wrote (in the learned form the gating after the candidate traversal also
// reads the upward pass's charges), so the upward pass runs on the context's
// side stream while the traversal runs on its stream, joined before the
// learned gating and before the evaluation (also under graph capture, where
// the fork and the join become edges of the graph).
stc_status do_upward_traverse(stc_ctx* c, const double* d_zeta, const double* d_area, bool stage_clock = false,
                              double t_off = 0.0) {
    if (c->n == 0) {
        stc_status st = do_upward(c, d_zeta, d_area, stage_clock, t_off);
        if (st == STC_OK) st = do_traverse(c);
        return st;
    }
    const stc_status sf = side_ready(c);
    if (sf != STC_OK) return sf;
    hipStream_t main = c->stream;
    if (hipEventRecord(c->ev_fork, main) != hipSuccess || hipStreamWaitEvent(c->side_stream, c->ev_fork, 0) != hipSuccess)
        return fail(c, STC_ERR_DEVICE, "stream fork failed");
    c->stream = c->side_stream;
    stc_status st = do_upward(c, d_zeta, d_area, stage_clock, t_off);
    c->stream = main;
    // the join is recorded and waited on whatever happened, so that a
    // capture stays well formed
    const bool joined = hipEventRecord(c->ev_join, c->side_stream) == hipSuccess;
    // the learned form's candidate traversal needs only the tree build; its
    // gating (features, network, resolve) waits for the upward pass
    c->gate_waits_upward = c->learned && joined;
    const stc_status st2 = do_traverse(c);
    c->gate_waits_upward = false;
    if (!joined || hipStreamWaitEvent(main, c->ev_join, 0) != hipSuccess)
        return fail(c, STC_ERR_DEVICE, "stream join failed");
    return st != STC_OK ? st : st2;
}

stc_status do_eval(stc_ctx* c, bool near, bool far, double* d_u, bool accumulate, bool stream = false) {
    if (c->n == 0) return STC_OK;
    hipStream_t s = c->stream;
    EvalArgs a = eval_args(c);
    a.stream = stream ? 1 : 0;
    u32 mask = (near ? 1u : 0u) | (far ? 2u : 0u);
    // near side, then the target-proxy values and their coefficients.  Running the
    // coefficients on the side stream beside k_near measured no faster: the two
    // kernels share the chip and each stretches by the other's time.
    phase_begin(c, 3);
    launch_near(s, a, mask);
    phase_end(c, 3);
    if (far) {
        phase_begin(c, 4);
        launch_far_targets(s, a);
        phase_end(c, 4);
    }
    phase_begin(c, 5);
    if (far) launch_far_finish(s, a);
    launch_l2p_finalize(s, a, far, d_u, accumulate);
    phase_end(c, 5);
    return check_launch(c, "eval");
}

stc_status check_ready(stc_ctx* c, bool need_lists) {
    if (!c) return STC_ERR_INVALID_ARG;
    if (!c->have_tree) return fail(c, STC_ERR_STATE, "no tree: call stc_tree_build first");
    if (need_lists && !(c->have_upward && c->have_lists))
        return fail(c, STC_ERR_STATE, "call stc_upward and stc_traverse before evaluating");
    return STC_OK;
}

// RK4 stage helpers ---------------------------------------------------------
__global__ void k_rk4_combine(i64 n, const double* __restrict__ x0, const double* __restrict__ z0,
                              const double* __restrict__ u, double omega, double c_next, double w_acc,
                              double* __restrict__ xs, double* __restrict__ zs, double* __restrict__ xacc,
                              double* __restrict__ zacc, int first) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double dz = -2.0 * omega * u[3 * i + 2];
    for (int c = 0; c < 3; ++c) {
        const double base = first ? x0[3 * i + c] : xacc[3 * i + c];
        xacc[3 * i + c] = base + w_acc * u[3 * i + c];
        xs[3 * i + c] = x0[3 * i + c] + c_next * u[3 * i + c];
    }
    const double zb = first ? z0[i] : zacc[i];
    zacc[i] = zb + w_acc * dz;
    zs[i] = z0[i] + c_next * dz;
}

__global__ void k_rk4_finish(i64 n, const double* __restrict__ xacc, const double* __restrict__ zacc,
                             double* __restrict__ x, double* __restrict__ z) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a = xacc[3 * i], b = xacc[3 * i + 1], cc = xacc[3 * i + 2];
    const double nr = sqrt((a * a + b * b) + cc * cc);
    x[3 * i] = a / nr;
    x[3 * i + 1] = b / nr;
    x[3 * i + 2] = cc / nr;
    z[i] = zacc[i];
}

// Sizes of a context's tables and buffers from its parameters (no device
// work, no host tables).
stc_status plan(stc_ctx* c, const stc_params* p, int32_t max_members, int64_t n_max_member, int64_t n_max_total) {
    stc_status st = validate_params(p, n_max_total);
    if (st != STC_OK) return st;
    if (max_members < 1 || max_members > STC_MAX_MEMBERS || n_max_member < 0 || n_max_member > n_max_total)
        return STC_ERR_INVALID_ARG;
    const bool learned = (p->flags & STC_FLAG_LEARNED) != 0;
    if (learned && max_members != 1) return STC_ERR_INVALID_ARG;
    const int L = p->max_level >= 0 ? p->max_level : stc_default_max_level(n_max_member, p->n_crit);
    const int mbits = bits_for(max_members);
    const int NB = std::max(1, bits_for(stc::total_nodes(L)));
    // leaf keys (member, face, 2L digits) are 32-bit; list keys hold two node ids and a type bit
    if (2 * L + 5 + mbits > 32 || NB + mbits > 31) return STC_ERR_INVALID_ARG;
    c->p = *p;
    c->n_max = n_max_total;
    c->n_max_member = n_max_member;
    c->max_members = max_members;
    c->L = L;
    c->p.max_level = c->L;
    c->np = stc_n_basis(p->degree);
    c->learned = learned;
    c->ndeg = learned ? 4 : 1;
    c->DB = learned ? 2 : 0;
    c->fb_class = learned ? (p->degree - 4) / 2 : 0;
    if (learned && !(c->p.theta_max > 0.0)) c->p.theta_max = p->theta;
    {
        int poff = 0, qoff = 0;
        for (int k = 0; k < 4; ++k) {
            const int d = learned ? 4 + 2 * k : (k == 0 ? p->degree : 0);
            const int np = k < c->ndeg ? stc_n_basis(d) : 0;
            c->cls.np[k] = np;
            c->cls.deg[k] = k < c->ndeg ? d : 0;
            c->cls.poff[k] = poff;
            c->cls.qoff[k] = qoff;
            poff += np;
            qoff += np * np;
        }
        c->NPT = poff;
    }
    c->NB = NB;
    c->LB = 2 * L + 5;
    c->n_local = stc::total_nodes(c->L);
    c->n_nodes = ((i64)(max_members - 1) << NB) + c->n_local;
    c->used_nodes = c->n_local;
    c->W = NB + mbits;
    // nodes with more than n_crit particles are disjoint within a level:
    // at most n_max / (n_crit + 1) per level over all members
    const i64 nm = std::max<i64>(n_max_total, 1);
    c->per_level = (u32)std::min<i64>(nm / (p->n_crit + 1) + 1, 0x7fffffffLL);
    c->slot_cap = (u32)std::min<i64>((i64)(c->L + 1) * c->per_level, 0x7fffffffLL);
    i64 cap = p->list_capacity > 0 ? p->list_capacity : std::max<i64>(65536, 16 * n_max_total);
    c->cap = (u32)std::min<i64>(cap, 0x7fffffffLL);
    // items: one per big node plus one per UP_CHUNK particles on each level
    c->items_cap = (u32)std::min<i64>((i64)c->slot_cap + (i64)(c->L + 1) * (nm / UP_CHUNK + 1), 0x7fffffffLL);
    c->hist_blocks = (int)((std::max<i64>(c->cap, nm) + 4095) / 4096);
    return STC_OK;
}

// Every device buffer of a context, in workspace order.
void carve(stc_ctx* c, Carver& cv) {
    const size_t nm = (size_t)std::max<i64>(c->n_max, 1), NPT = (size_t)c->NPT, ns = c->slot_cap;
    const size_t ngeo = (size_t)stc::total_nodes(c->L), nnodes = (size_t)c->n_nodes;
    size_t nq = 0;
    for (int k = 0; k < c->ndeg; ++k) nq += (size_t)c->cls.np[k] * c->cls.np[k];
    const size_t nseg = nnodes << c->DB;
    cv.take(&c->geo, ngeo);
    cv.take(&c->mac, ngeo);
    cv.take(&c->ncnt, nnodes);
    cv.take(&c->slot, nnodes);
    cv.take(&c->big_list, (size_t)(c->L + 1) * c->per_level);
    cv.take(&c->level_off, (size_t)c->L + 2);
    cv.take(&c->ref_points, 3 * NPT);
    cv.take(&c->ref_vinv, nq);
    cv.take(&c->ref_vinvT, nq);
    cv.take(&c->ref_coef, NPT);
    cv.take(&c->ref_expo, 3 * NPT);
    cv.take(&c->keys_a, nm);
    cv.take(&c->keys_b, nm);
    cv.take(&c->perm, nm);
    cv.take(&c->leaf, nm);
    cv.take(&c->sx, nm);
    cv.take(&c->sy, nm);
    cv.take(&c->sz, nm);
    cv.take(&c->sq, nm);
    cv.take(&c->nbeg, nnodes);
    cv.take(&c->nend, nnodes);
    cv.take(&c->prox, ns * NPT);
    cv.take(&c->alpha, ns * NPT * 3);
    cv.take(&c->Wacc, 3 * nm);
    cv.take(&c->front0, c->cap);
    cv.take(&c->front1, c->cap);
    cv.take(&c->tlist_a, c->cap);
    cv.take(&c->tlist_b, c->cap);
    cv.take(&c->nlist_a, c->cap);
    cv.take(&c->nlist_b, c->cap);
    cv.take(&c->tseg_beg, nnodes);
    cv.take(&c->tseg_end, nnodes);
    cv.take(&c->nseg_beg, nseg);
    cv.take(&c->nseg_end, nseg);
    cv.take(&c->counters, C_COUNT);
    cv.take(&c->flags, F_COUNT);
    cv.take(&c->evals, 8);
    cv.take(&c->sort_zero, kSortZeroWords);
    cv.take(&c->sort_status, (size_t)2 * 256 * c->hist_blocks);
    cv.take(&c->sort_epoch, 2);
    cv.take(&c->rk_x, 3 * nm);
    cv.take(&c->rk_z, nm);
    cv.take(&c->rk_u, 3 * nm);
    cv.take(&c->rk_xacc, 3 * nm);
    cv.take(&c->rk_zacc, nm);
    cv.take(&c->forcing_t, 1);
    cv.take(&c->item_node, c->items_cap);
    cv.take(&c->item_chunk, c->items_cap);
    cv.take(&c->item_base, ns);
    cv.take(&c->upart, (size_t)c->items_cap * c->cls.np[c->ndeg - 1]);
    if (c->learned) {
        cv.take(&c->ref_T, (size_t)c->cls.poff[3] * c->cls.np[3]);
        cv.take(&c->up_T, (size_t)c->cls.poff[3] * c->cls.np[3]);
        cv.take(&c->up_H, (size_t)c->cls.np[3] * c->cls.np[3]);
        cv.take(&c->cls_mask, c->slot_cap);
        cv.take(&c->cand, c->cap);
        cv.take(&c->feat, (size_t)c->cap * 16);
        cv.take(&c->mlp_out, (size_t)c->cap * 4);
        cv.take(&c->qabs, nnodes);
        cv.take(&c->qsum, nnodes);
    }
}

}  // namespace

// Scratch of stc_direct_noalloc: the source chunks' partial sums
// (chunks x m x 3 doubles) live in this file-scope array instead of a
// stream-ordered allocation.  Each GPU holds its own copy from the first
// call on it until the process ends.  In host code `scratch` only names the
// symbol: its device address comes from hipGetSymbolAddress, taken once per
// device and kept in g_scratch_addr.
constexpr size_t kNoAllocScratchBytes = (size_t)16 << 20;
constexpr int kMaxScratchDevices = 64;
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

namespace {
std::mutex g_scratch_mu;
double* g_scratch_addr[kMaxScratchDevices] = {};

// Device address of the current device's scratch array (set up on the first
// call on that device, with that device current).
stc_status noalloc_scratch(double** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxScratchDevices) return STC_ERR_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return STC_ERR_DEVICE;
        }
        g_scratch_addr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_addr[dev];
    return STC_OK;
}

// Where the chunk partial sums of a split direct sum go.
enum class DirectScratch { Caller, Static };

// Source chunks of a direct sum of m targets over n sources on the current
// device and the bytes of their partial sums (0 when unsplit).
stc_status direct_plan(i64 n, i64 m, int32_t precision, int32_t denominator, u32* chunks, i64* chunk_len,
                       size_t* bytes) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess)
        return STC_ERR_DEVICE;
    direct_split(n, m, cus, direct_blocks_per_cu(precision, denominator), direct_targets_per_block(precision), chunks,
                 chunk_len);
    *bytes = *chunks > 1 ? (size_t)*chunks * (size_t)m * 3 * sizeof(double) : 0;
    return STC_OK;
}
}  // namespace

extern "C" {

const char* stc_status_string(int32_t status) {
    if (status < 0 || status > 7) return "unknown status";
    return kStatusText[status];
}

stc_status stc_default_params(stc_params* p) {
    if (!p) return STC_ERR_INVALID_ARG;
    std::memset(p, 0, sizeof(*p));
    p->theta = 0.7;
    p->degree = 8;
    p->n_crit = 64;
    p->max_level = -1;
    p->precision = STC_FP64;
    p->denominator = STC_DEN_DOT;
    p->list_capacity = 0;
    return STC_OK;
}

int32_t stc_n_basis(int32_t degree) {
    if (degree < 1 || degree > kMaxDegree) return 0;
    return (degree + 1) * (degree + 2) / 2;
}

int64_t stc_total_nodes(int32_t max_level) {
    if (max_level < 0 || max_level > 12) return 0;
    return stc::total_nodes(max_level);
}

int32_t stc_default_max_level(int64_t n_max, int32_t n_crit) {
    if (n_crit < 1) n_crit = 1;
    int lvl = 0;
    while ((i64)20 * ((i64)1 << (2 * lvl)) * n_crit < n_max && lvl < 30) ++lvl;
    return std::min(12, lvl + 2);
}

stc_status stc_create(const stc_params* p, int64_t n_max, void* d_ws, size_t ws_bytes, void* hip_stream,
                      stc_ctx** out) {
    return stc_create_batched(p, 1, n_max, n_max, d_ws, ws_bytes, hip_stream, out);
}

stc_status stc_workspace_size(const stc_params* p, int64_t n_max, size_t* bytes) {
    return stc_workspace_size_batched(p, 1, n_max, n_max, bytes);
}

stc_status stc_workspace_size_batched(const stc_params* p, int32_t max_members, int64_t n_max_member,
                                      int64_t n_max_total, size_t* bytes) {
    if (!bytes) return STC_ERR_INVALID_ARG;
    *bytes = 0;
    stc_ctx* c = new (std::nothrow) stc_ctx();
    if (!c) return STC_ERR_ALLOC;
    stc_status st = plan(c, p, max_members, n_max_member, n_max_total);
    if (st == STC_OK) {
        Carver cv;
        carve(c, cv);
        *bytes = cv.off;
    }
    delete c;
    return st;
}

stc_status stc_create_batched(const stc_params* p, int32_t max_members, int64_t n_max_member, int64_t n_max_total,
                              void* d_ws, size_t ws_bytes, void* hip_stream, stc_ctx** out) {
    if (!out) return STC_ERR_INVALID_ARG;
    *out = nullptr;
    stc_ctx* c = new (std::nothrow) stc_ctx();
    if (!c) return STC_ERR_ALLOC;
    stc_status st = plan(c, p, max_members, n_max_member, n_max_total);
    if (st != STC_OK) {
        delete c;
        return st;
    }
    {
        Carver cv;
        carve(c, cv);
        if (!d_ws || (reinterpret_cast<uintptr_t>(d_ws) & (kWorkspaceAlign - 1)) || ws_bytes < cv.off) {
            delete c;
            return STC_ERR_WORKSPACE;
        }
        cv = Carver{static_cast<char*>(d_ws), 0};
        carve(c, cv);
        c->ws = d_ws;
        c->ws_bytes = ws_bytes;
    }
    c->stream = static_cast<hipStream_t>(hip_stream);
    try {
        build_tree_geometry(c->L, c->geo_host);
        for (int k = 0; k < c->ndeg; ++k)
            if (!build_reference_tables(c->cls.deg[k], c->ref_host[k])) {
                delete c;
                return STC_ERR_INVALID_ARG;
            }
    } catch (...) {
        delete c;
        return STC_ERR_ALLOC;
    }
    c->level_off_host.resize(c->L + 2);
    for (int l = 0; l <= c->L + 1; ++l) c->level_off_host[l] = level_offset(l);
    c->tlist = c->tlist_a;
    c->nlist = c->nlist_a;
    hipStream_t s = c->stream;
    // all classes' tables, concatenated (class k at poff[k] points, qoff[k] matrix entries)
    std::vector<double> pts_h, vinv_h, vinvT_h, coef_h;
    std::vector<int> expo_h;
    for (int k = 0; k < c->ndeg; ++k) {
        const RefTables& t = c->ref_host[k];
        const size_t n = (size_t)t.np;
        pts_h.insert(pts_h.end(), t.points.begin(), t.points.end());
        vinv_h.insert(vinv_h.end(), t.vinv.begin(), t.vinv.end());
        for (size_t m = 0; m < n; ++m)
            for (size_t kk = 0; kk < n; ++kk) vinvT_h.push_back(t.vinv[kk * n + m]);
        coef_h.insert(coef_h.end(), t.coef.begin(), t.coef.end());
        expo_h.insert(expo_h.end(), t.expo.begin(), t.expo.end());
    }
    std::vector<NodeMac> mac_host(c->geo_host.size());
    for (size_t i = 0; i < mac_host.size(); ++i)
        mac_host[i] = NodeMac{c->geo_host[i].c[0], c->geo_host[i].c[1], c->geo_host[i].c[2], c->geo_host[i].r};
    auto up = [&](void* dst, const void* src, size_t bytes) {
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) == hipSuccess;
    };
    bool cp = up(c->geo, c->geo_host.data(), c->geo_host.size() * sizeof(NodeGeo)) &&
              up(c->mac, mac_host.data(), mac_host.size() * sizeof(NodeMac)) &&
              up(c->level_off, c->level_off_host.data(), c->level_off_host.size() * sizeof(i64)) &&
              up(c->ref_points, pts_h.data(), pts_h.size() * sizeof(double)) &&
              up(c->ref_vinv, vinv_h.data(), vinv_h.size() * sizeof(double)) &&
              up(c->ref_vinvT, vinvT_h.data(), vinvT_h.size() * sizeof(double)) &&
              up(c->ref_coef, coef_h.data(), coef_h.size() * sizeof(double)) &&
              up(c->ref_expo, expo_h.data(), expo_h.size() * sizeof(int));
    // sort look-back statuses and epochs start cleared (a status matches only
    // the epoch of the pass that wrote it; epochs start at 1)
    cp = cp && hipMemsetAsync(c->sort_status, 0, (size_t)2 * 256 * c->hist_blocks * sizeof(u64), s) == hipSuccess &&
         hipMemsetAsync(c->sort_epoch, 0, 2 * sizeof(u32), s) == hipSuccess;
    // learned form, in long double:
    //   T[n * 88 + poff_c + m] = sum_k (V_ref,d^{-1})_km B_k(b_10,n): class c's
    //     Lagrange basis at the degree-10 reference points (degree-10 point
    //     charges -> degree d in the upward pass; kept transposed as well,
    //     [(poff_c + m) * 66 + n], for the far field's values -> degree 10);
    //   H[n * 66 + k] = c_k (V_ref,10^{-1})_kn: degree-10 coefficients (times
    //     their multinomials, as stored) from values at the degree-10 points
    std::vector<double> T_h, Tu_h, H_h;
    if (c->learned) {
        const RefTables& t10 = c->ref_host[3];
        const int nout = c->cls.poff[3];
        T_h.assign((size_t)t10.np * nout, 0.0);
        Tu_h.assign((size_t)nout * t10.np, 0.0);
        for (int k = 0; k < 3; ++k) {
            const RefTables& td = c->ref_host[k];
            for (int m = 0; m < td.np; ++m)
                for (int n = 0; n < t10.np; ++n) {
                    long double acc = 0.0L;
                    for (int kk = 0; kk < td.np; ++kk) {
                        long double B = td.coef[kk];
                        for (int a = 0; a < 3; ++a)
                            for (int e = 0; e < td.expo[3 * kk + a]; ++e) B *= (long double)t10.points[3 * n + a];
                        acc += (long double)td.vinv[(size_t)kk * td.np + m] * B;
                    }
                    T_h[(size_t)n * nout + c->cls.poff[k] + m] = (double)acc;
                    Tu_h[(size_t)(c->cls.poff[k] + m) * t10.np + n] = (double)acc;
                }
        }
        H_h.assign((size_t)t10.np * t10.np, 0.0);
        for (int n = 0; n < t10.np; ++n)
            for (int kk = 0; kk < t10.np; ++kk)
                H_h[(size_t)n * t10.np + kk] =
                    (double)((long double)t10.coef[kk] * (long double)t10.vinv[(size_t)kk * t10.np + n]);
        cp = cp && up(c->ref_T, T_h.data(), T_h.size() * sizeof(double)) &&
             up(c->up_T, Tu_h.data(), Tu_h.size() * sizeof(double)) &&
             up(c->up_H, H_h.data(), H_h.size() * sizeof(double));
    }
    launch_fill_u32(s, c->counters, C_COUNT, 0u);
    launch_fill_u32(s, c->flags, F_COUNT, 0u);
    if (!cp || hipStreamSynchronize(s) != hipSuccess) {
        stc_destroy(c);
        return STC_ERR_DEVICE;
    }
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
            c->cus = prop.multiProcessorCount;
    }
    c->shape_default = stc_launch_config{256, 48, 256, 48};
    *out = c;
    return STC_OK;
}

stc_status stc_destroy(stc_ctx* c) {
    if (!c) return STC_ERR_INVALID_ARG;
    (void)hipStreamSynchronize(c->stream);
    rk4_drop_graph(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->side_stream) {
        (void)hipStreamSynchronize(c->side_stream);
        (void)hipStreamDestroy(c->side_stream);
    }
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
    delete c;
    return STC_OK;
}

stc_status stc_set_stream(stc_ctx* c, void* hip_stream) {
    if (!c) return STC_ERR_INVALID_ARG;
    c->stream = static_cast<hipStream_t>(hip_stream);
    return STC_OK;
}

stc_status stc_get_params(const stc_ctx* c, stc_params* out) {
    if (!c || !out) return STC_ERR_INVALID_ARG;
    *out = c->p;
    return STC_OK;
}

stc_status stc_tree_build(stc_ctx* c, int64_t n, const double* d_x) {
    if (!c) return STC_ERR_INVALID_ARG;
    if (n < 0 || n > c->n_max) return fail(c, STC_ERR_INVALID_ARG, "n out of range [0, n_max]");
    if (n > 0 && (!d_x || !aligned8(d_x))) return fail(c, STC_ERR_INVALID_ARG, "d_x is NULL or misaligned");
    const i64 off[2] = {0, n};
    return do_build(c, 1, off, d_x);
}

stc_status stc_tree_build_batched(stc_ctx* c, int32_t members, const int64_t* h_offsets, const double* d_x) {
    if (!c) return STC_ERR_INVALID_ARG;
    const i64 n = check_offsets(c, members, h_offsets);
    if (n < 0) return fail(c, STC_ERR_INVALID_ARG, "bad member count or offsets");
    if (n > 0 && (!d_x || !aligned8(d_x))) return fail(c, STC_ERR_INVALID_ARG, "d_x is NULL or misaligned");
    return do_build(c, members, h_offsets, d_x);
}

stc_status stc_upward(stc_ctx* c, const double* d_zeta, const double* d_area) {
    stc_status st = check_ready(c, false);
    if (st != STC_OK) return st;
    if (c->n > 0 && (!d_zeta || !d_area || !aligned8(d_zeta) || !aligned8(d_area)))
        return fail(c, STC_ERR_INVALID_ARG, "d_zeta / d_area NULL or misaligned");
    return do_upward(c, d_zeta, d_area);
}

stc_status stc_traverse(stc_ctx* c) {
    stc_status st = check_ready(c, false);
    if (st != STC_OK) return st;
    return do_traverse(c);
}

stc_status stc_eval_near(stc_ctx* c, double* d_u, int32_t accumulate) {
    stc_status st = check_ready(c, true);
    if (st != STC_OK) return st;
    if (c->n > 0 && (!d_u || !aligned8(d_u))) return fail(c, STC_ERR_INVALID_ARG, "d_u NULL or misaligned");
    return do_eval(c, true, false, d_u, accumulate != 0);
}

stc_status stc_eval_far(stc_ctx* c, double* d_u, int32_t accumulate) {
    stc_status st = check_ready(c, true);
    if (st != STC_OK) return st;
    if (c->n > 0 && (!d_u || !aligned8(d_u))) return fail(c, STC_ERR_INVALID_ARG, "d_u NULL or misaligned");
    return do_eval(c, false, true, d_u, accumulate != 0);
}

stc_status stc_velocity(stc_ctx* c, int64_t n, const double* d_x, const double* d_zeta, const double* d_area,
                        double* d_u) {
    if (!c) return STC_ERR_INVALID_ARG;
    if (n < 0 || n > c->n_max) return fail(c, STC_ERR_INVALID_ARG, "n out of range [0, n_max]");
    if (n > 0 && (!d_x || !d_zeta || !d_area || !d_u || !aligned8(d_x) || !aligned8(d_zeta) || !aligned8(d_area) ||
                  !aligned8(d_u)))
        return fail(c, STC_ERR_INVALID_ARG, "NULL or misaligned pointer");
    const i64 off[2] = {0, n};
    stc_status st = do_build(c, 1, off, d_x);
    if (st == STC_OK) st = do_upward_traverse(c, d_zeta, d_area);
    if (st == STC_OK) st = do_eval(c, true, true, d_u, false);
    return st;
}

stc_status stc_velocity_batched(stc_ctx* c, int32_t members, const int64_t* h_offsets, const double* d_x,
                                const double* d_zeta, const double* d_area, double* d_u) {
    if (!c) return STC_ERR_INVALID_ARG;
    const i64 n = check_offsets(c, members, h_offsets);
    if (n < 0) return fail(c, STC_ERR_INVALID_ARG, "bad member count or offsets");
    if (n > 0 && (!d_x || !d_zeta || !d_area || !d_u || !aligned8(d_x) || !aligned8(d_zeta) || !aligned8(d_area) ||
                  !aligned8(d_u)))
        return fail(c, STC_ERR_INVALID_ARG, "NULL or misaligned pointer");
    stc_status st = do_build(c, members, h_offsets, d_x);
    if (st == STC_OK) st = do_upward_traverse(c, d_zeta, d_area);
    if (st == STC_OK) st = do_eval(c, true, true, d_u, false);
    return st;
}

static stc_status direct_check(int64_t n, int64_t m, int32_t precision, int32_t denominator) {
    if (n < 0 || m < 0 || n >= 0x7fffffffLL) return STC_ERR_INVALID_ARG;
    if (precision != STC_FP64 && precision != STC_FP32) return STC_ERR_INVALID_ARG;
    if (denominator != STC_DEN_DOT && denominator != STC_DEN_DIST2) return STC_ERR_INVALID_ARG;
    if (precision == STC_FP32 && denominator != STC_DEN_DIST2) return STC_ERR_INVALID_ARG;
    return STC_OK;
}

static stc_status direct_sum(void* hip_stream, int64_t n, const double* d_x, const double* d_zeta,
                             const double* d_area, int64_t m, const int64_t* d_targets, int32_t precision,
                             int32_t denominator, double* d_u, bool stream, DirectScratch where, void* d_scratch,
                             size_t scratch_bytes) {
    stc_status st = direct_check(n, m, precision, denominator);
    if (st != STC_OK) return st;
    if (!d_targets && m != n) return STC_ERR_INVALID_ARG;
    if (m == 0) return STC_OK;
    if (n == 0 || !d_x || !d_zeta || !d_area || !d_u || !aligned8(d_x) || !aligned8(d_zeta) || !aligned8(d_area) ||
        !aligned8(d_u) || (d_targets && !aligned8(d_targets)))
        return STC_ERR_INVALID_ARG;
    // Few targets cannot fill the chip: the sources are split into chunks
    // whose partial sums go to the caller's scratch (or, for the
    // no-allocation form, the static scratch array) and are added in chunk
    // order by a second kernel.
    u32 chunks = 1;
    i64 chunk_len = n;
    size_t bytes = 0;
    st = direct_plan(n, m, precision, denominator, &chunks, &chunk_len, &bytes);
    if (st != STC_OK) return st;
    double* part = nullptr;
    if (bytes > 0 && where == DirectScratch::Static) {
        if (bytes > kNoAllocScratchBytes) return STC_ERR_WORKSPACE;
        st = noalloc_scratch(&part);
        if (st != STC_OK) return st;
    } else if (bytes > 0) {
        if (!d_scratch || !aligned8(d_scratch) || scratch_bytes < bytes) return STC_ERR_WORKSPACE;
        part = static_cast<double*>(d_scratch);
    }
    launch_direct(static_cast<hipStream_t>(hip_stream), n, d_x, d_zeta, d_area, m, d_targets, precision, denominator,
                  chunks, chunk_len, part, d_u, stream ? 1 : 0);
    return hipGetLastError() == hipSuccess ? STC_OK : STC_ERR_DEVICE;
}

stc_status stc_direct_scratch_size(int64_t n, int64_t m, int32_t precision, int32_t denominator, size_t* bytes) {
    if (!bytes) return STC_ERR_INVALID_ARG;
    *bytes = 0;
    stc_status st = direct_check(n, m, precision, denominator);
    if (st != STC_OK || n == 0 || m == 0) return st;
    u32 chunks = 1;
    i64 chunk_len = n;
    return direct_plan(n, m, precision, denominator, &chunks, &chunk_len, bytes);
}

stc_status stc_direct(void* hip_stream, int64_t n, const double* d_x, const double* d_zeta, const double* d_area,
                      int64_t m, const int64_t* d_targets, int32_t precision, int32_t denominator, double* d_u,
                      void* d_scratch, size_t scratch_bytes) {
    return direct_sum(hip_stream, n, d_x, d_zeta, d_area, m, d_targets, precision, denominator, d_u, false,
                      DirectScratch::Caller, d_scratch, scratch_bytes);
}

stc_status stc_direct_noalloc(void* hip_stream, int64_t n, const double* d_x, const double* d_zeta,
                              const double* d_area, int64_t m, const int64_t* d_targets, int32_t precision,
                              int32_t denominator, double* d_u) {
    return direct_sum(hip_stream, n, d_x, d_zeta, d_area, m, d_targets, precision, denominator, d_u, false,
                      DirectScratch::Static, nullptr, 0);
}

stc_status stc_direct_stream(void* hip_stream, int64_t n, const double* d_x, const double* d_zeta,
                             const double* d_area, int64_t m, const int64_t* d_targets, int32_t precision,
                             int32_t denominator, double* d_psi, void* d_scratch, size_t scratch_bytes) {
    return direct_sum(hip_stream, n, d_x, d_zeta, d_area, m, d_targets, precision, denominator, d_psi, true,
                      DirectScratch::Caller, d_scratch, scratch_bytes);
}

stc_status stc_stream_function(stc_ctx* c, int64_t n, const double* d_x, const double* d_zeta, const double* d_area,
                               double* d_psi) {
    if (!c) return STC_ERR_INVALID_ARG;
    if (c->learned) return fail(c, STC_ERR_INVALID_ARG, "the learned form gates velocity interactions only");
    if (n < 0 || n > c->n_max) return fail(c, STC_ERR_INVALID_ARG, "n out of range [0, n_max]");
    if (n > 0 && (!d_x || !d_zeta || !d_area || !d_psi || !aligned8(d_x) || !aligned8(d_zeta) ||
                  !aligned8(d_area) || !aligned8(d_psi)))
        return fail(c, STC_ERR_INVALID_ARG, "NULL or misaligned pointer");
    const i64 off[2] = {0, n};
    stc_status st = do_build(c, 1, off, d_x);
    if (st == STC_OK) st = do_upward_traverse(c, d_zeta, d_area);
    if (st == STC_OK) st = do_eval(c, true, true, d_psi, false, true);
    return st;
}

stc_status stc_stream_function_batched(stc_ctx* c, int32_t members, const int64_t* h_offsets, const double* d_x,
                                       const double* d_zeta, const double* d_area, double* d_psi) {
    if (!c) return STC_ERR_INVALID_ARG;
    if (c->learned) return fail(c, STC_ERR_INVALID_ARG, "the learned form gates velocity interactions only");
    const i64 n = check_offsets(c, members, h_offsets);
    if (n < 0) return fail(c, STC_ERR_INVALID_ARG, "bad member count or offsets");
    if (n > 0 && (!d_x || !d_zeta || !d_area || !d_psi || !aligned8(d_x) || !aligned8(d_zeta) ||
                  !aligned8(d_area) || !aligned8(d_psi)))
        return fail(c, STC_ERR_INVALID_ARG, "NULL or misaligned pointer");
    stc_status st = do_build(c, members, h_offsets, d_x);
    if (st == STC_OK) st = do_upward_traverse(c, d_zeta, d_area);
    if (st == STC_OK) st = do_eval(c, true, true, d_psi, false, true);
    return st;
}

// Enqueues one RK4 step of every member on c->stream (no host
// synchronisation, no memsets).
static stc_status rk4_enqueue_step(stc_ctx* c, int members, const i64* off, double* d_x, double* d_zeta,
                                   const double* d_area, double dt, double omega) {
    hipStream_t s = c->stream;
    const i64 n = off[members];
    const dim3 g((unsigned)((n + 255) / 256)), b(256);
    // stage nodes 0, 1/2, 1/2, 1; weights 1/6, 1/3, 1/3, 1/6
    const double cnext[4] = {0.5 * dt, 0.5 * dt, dt, 0.0};
    const double wacc[4] = {dt / 6.0, dt / 3.0, dt / 3.0, dt / 6.0};
    const double stage_t[4] = {0.0, 0.5 * dt, 0.5 * dt, dt};  // forcing time of each stage after the step's start
    const double* xs = d_x;
    const double* zs = d_zeta;
    for (int stg = 0; stg < 4; ++stg) {
        stc_status st = do_build(c, members, off, xs);
        if (st == STC_OK) st = do_upward_traverse(c, zs, d_area, true, stage_t[stg]);
        if (st == STC_OK) st = do_eval(c, true, true, c->rk_u, false);
        if (st != STC_OK) return st;
        hipLaunchKernelGGL(k_rk4_combine, g, b, 0, s, (i64)n, d_x, d_zeta, c->rk_u, omega, cnext[stg], wacc[stg],
                           c->rk_x, c->rk_z, c->rk_xacc, c->rk_zacc, stg == 0 ? 1 : 0);
        xs = c->rk_x;
        zs = c->rk_z;
    }
    hipLaunchKernelGGL(k_rk4_finish, g, b, 0, s, (i64)n, c->rk_xacc, c->rk_zacc, d_x, d_zeta);
    if (c->forcing_on) launch_forcing_clock(s, c->forcing_t, dt, 0);
    return check_launch(c, "rk4");
}

static void rk4_drop_graph(stc_ctx* c) {
    if (c->rk_exec) (void)hipGraphExecDestroy(c->rk_exec);
    c->rk_exec = nullptr;
    c->rk_n = -1;
    c->rk_offsets.clear();
}

// Captures one RK4 step into a graph (on the context's capture stream).
static stc_status rk4_capture(stc_ctx* c, int members, const i64* off, double* d_x, double* d_zeta,
                              const double* d_area, double dt, double omega) {
    rk4_drop_graph(c);
    if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return fail(c, STC_ERR_DEVICE, "creating the capture stream failed");
    // the capture must not record timing events
    const int tmax = c->t_max;
    c->t_max = 0;
    hipStream_t user = c->stream;
    c->stream = c->cap_stream;
    hipGraph_t graph = nullptr;
    stc_status st = STC_OK;
    if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        st = fail(c, STC_ERR_DEVICE, "hipStreamBeginCapture failed");
    } else {
        st = rk4_enqueue_step(c, members, off, d_x, d_zeta, d_area, dt, omega);
        const hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
        if (st == STC_OK && e != hipSuccess) st = fail(c, STC_ERR_DEVICE, "hipStreamEndCapture failed");
    }
    c->stream = user;
    c->t_max = tmax;
    if (st == STC_OK && hipGraphInstantiate(&c->rk_exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        c->rk_exec = nullptr;
        st = fail(c, STC_ERR_DEVICE, "hipGraphInstantiate failed");
    }
    if (graph) (void)hipGraphDestroy(graph);
    if (st != STC_OK) return st;
    c->rk_n = off[members];
    c->rk_offsets.assign(off, off + members + 1);
    c->rk_px = d_x;
    c->rk_pz = d_zeta;
    c->rk_pa = d_area;
    c->rk_dt = dt;
    c->rk_om = omega;
    return STC_OK;
}

static stc_status rk4_run(stc_ctx* c, int members, const i64* off, double* d_x, double* d_zeta,
                          const double* d_area, double dt, double omega, int32_t n_steps, bool eager = false) {
    const i64 n = off[members];
    if (n_steps < 0 || !std::isfinite(dt) || !std::isfinite(omega))
        return fail(c, STC_ERR_INVALID_ARG, "bad n_steps, dt or omega");
    if (n == 0 || n_steps == 0) {
        if (c->forcing_on) c->forcing.time += (double)n_steps * dt;
        return STC_OK;
    }
    if (!d_x || !d_zeta || !d_area || !aligned8(d_x) || !aligned8(d_zeta) || !aligned8(d_area))
        return fail(c, STC_ERR_INVALID_ARG, "NULL or misaligned pointer");
    // RK4 stage points leave the sphere (|x_s| - 1 ~ (dt |u|)^2 / 8); 1 - x.y can
    // then vanish or turn negative for close pairs, |x - y|^2 / 2 cannot
    if (c->p.denominator != STC_DEN_DIST2)
        return fail(c, STC_ERR_INVALID_ARG, "stc_rk4 needs the |x-y|^2/2 denominator (stage points are off the sphere)");
    const bool use_graph = !eager && (c->p.flags & STC_FLAG_EAGER_RK4) == 0;
    // the steps read their start time from the device clock (a kernel, not a
    // memset: the clock is also written inside captured steps)
    if (c->forcing_on) launch_forcing_clock(c->stream, c->forcing_t, c->forcing.time, 1);
    if (!use_graph) {
        for (int step = 0; step < n_steps; ++step) {
            stc_status st = rk4_enqueue_step(c, members, off, d_x, d_zeta, d_area, dt, omega);
            if (st != STC_OK) return st;
        }
    } else {
        const bool same = c->rk_exec && c->rk_n == n && c->rk_px == d_x && c->rk_pz == d_zeta &&
                          c->rk_pa == d_area && c->rk_dt == dt && c->rk_om == omega &&
                          c->rk_offsets.size() == (size_t)members + 1 &&
                          std::equal(c->rk_offsets.begin(), c->rk_offsets.end(), off);
        if (!same) {
            stc_status st = rk4_capture(c, members, off, d_x, d_zeta, d_area, dt, omega);
            if (st != STC_OK) return st;
        }
        for (int step = 0; step < n_steps; ++step)
            if (hipGraphLaunch(c->rk_exec, c->stream) != hipSuccess)
                return fail(c, STC_ERR_DEVICE, "hipGraphLaunch failed");
    }
    c->have_tree = c->have_upward = c->have_lists = false;  // stage data, not the final state
    if (c->forcing_on) c->forcing.time += (double)n_steps * dt;
    return STC_OK;
}

stc_status stc_set_forcing(stc_ctx* c, const stc_forcing* f) {
    if (!c) return STC_ERR_INVALID_ARG;
    if (f) {
        if (!forcing_valid(f))
            return fail(c, STC_ERR_INVALID_ARG, "forcing needs 0 <= k <= 16, 0 < lat1 < pi/2, T_p > 0, T_f >= 2 T_p");
        c->forcing = *f;
    }
    c->forcing_on = f != nullptr;
    rk4_drop_graph(c);
    return STC_OK;
}

stc_status stc_forcing_field(void* hip_stream, const stc_forcing* f, int64_t n, const double* d_x, double* d_out) {
    if (!f || !forcing_valid(f) || n < 0 || (n > 0 && (!d_x || !d_out || !aligned8(d_x) || !aligned8(d_out))))
        return STC_ERR_INVALID_ARG;
    if (n == 0) return STC_OK;
    launch_forcing_field(static_cast<hipStream_t>(hip_stream), n, d_x, forcing_dev(*f, f->time, nullptr), d_out);
    return hipGetLastError() == hipSuccess ? STC_OK : STC_ERR_DEVICE;
}

stc_status stc_get_forcing(const stc_ctx* c, stc_forcing* f, int32_t* on) {
    if (!c) return STC_ERR_INVALID_ARG;
    if (f) *f = c->forcing;
    if (on) *on = c->forcing_on ? 1 : 0;
    return STC_OK;
}

stc_status stc_rk4(stc_ctx* c, int64_t n, double* d_x, double* d_zeta, const double* d_area, double dt, double omega,
                   int32_t n_steps) {
    if (!c) return STC_ERR_INVALID_ARG;
    if (n < 0 || n > c->n_max) return fail(c, STC_ERR_INVALID_ARG, "n out of range [0, n_max]");
    const i64 off[2] = {0, n};
    return rk4_run(c, 1, off, d_x, d_zeta, d_area, dt, omega, n_steps);
}

stc_status stc_rk4_batched(stc_ctx* c, int32_t members, const int64_t* h_offsets, double* d_x, double* d_zeta,
                           const double* d_area, double dt, double omega, int32_t n_steps) {
    if (!c) return STC_ERR_INVALID_ARG;
    if (check_offsets(c, members, h_offsets) < 0) return fail(c, STC_ERR_INVALID_ARG, "bad member count or offsets");
    return rk4_run(c, members, h_offsets, d_x, d_zeta, d_area, dt, omega, n_steps);
}

stc_status stc_amr_rk4(stc_amr* m, stc_ctx* c, double dt, double omega, int32_t n_steps) {
    if (!m || !c) return STC_ERR_INVALID_ARG;
    if (n_steps < 0) return fail(c, STC_ERR_INVALID_ARG, "n_steps < 0");
    if (amr_stream(m) != c->stream) return fail(c, STC_ERR_INVALID_ARG, "the mesh and the context use different streams");
    if (c->learned || c->members != 1) return fail(c, STC_ERR_INVALID_ARG, "a single-member context without gating");
    for (int step = 0; step < n_steps; ++step) {
        int64_t n = 0;
        double *x = nullptr, *z = nullptr, *a = nullptr;
        stc_status st = stc_amr_particles(m, &n, &x, &z, &a);
        if (st != STC_OK) return st;
        if (n > c->n_max) return fail(c, STC_ERR_CAPACITY, "the mesh has more particles than the context holds");
        const i64 off[2] = {0, n};
        st = rk4_run(c, 1, off, x, z, a, dt, omega, 1, true);
        if (st == STC_OK) st = stc_amr_set_state(m, n, x, z);
        if (st == STC_OK) st = stc_amr_adapt(m);
        if (st != STC_OK) return st;
    }
    return STC_OK;
}

stc_status stc_node_layout(const stc_ctx* c, int32_t* node_bits, int64_t* nodes_per_member, int64_t* node_array_len) {
    if (!c) return STC_ERR_INVALID_ARG;
    if (node_bits) *node_bits = c->NB;
    if (nodes_per_member) *nodes_per_member = c->n_local;
    if (node_array_len) *node_array_len = c->n_nodes;
    return STC_OK;
}

stc_status stc_get_launch_config(const stc_ctx* c, int64_t n_total, stc_launch_config* out) {
    if (!c || !out) return STC_ERR_INVALID_ARG;
    *out = shape_for(c, n_total);
    return STC_OK;
}

stc_status stc_set_launch_config(stc_ctx* c, int64_t n_total, const stc_launch_config* cfg) {
    if (!c || !valid_shape(cfg)) return STC_ERR_INVALID_ARG;
    if (n_total < 0) c->shape_default = *cfg;
    else c->shapes[size_class(n_total)] = *cfg;
    return STC_OK;
}

stc_status stc_autotune(stc_ctx* c, int32_t repeats, stc_launch_config* out) {
    stc_status st = check_ready(c, true);
    if (st != STC_OK) return st;
    if (repeats < 1 || repeats > 100 || !out) return fail(c, STC_ERR_INVALID_ARG, "repeats must be in [1, 100]");
    st = stc_sync(c);
    if (st != STC_OK) return st;
    stc_launch_config best = shape_for(c, c->n);
    if (c->n == 0) {
        *out = best;
        return STC_OK;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(c, STC_ERR_DEVICE, "hipEventCreate failed");
    }
    hipStream_t s = c->stream;
    EvalArgs a = eval_args(c);
    bool ok = true;
    auto timed = [&](auto launch) -> float {
        launch();  // warm-up
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < repeats; ++r) launch();
        (void)hipEventRecord(e1, s);
        float ms = 0.f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) ok = false;
        return ms / repeats;
    };
    const int threads[3] = {128, 256, 512};
    const int per_cu[6] = {8, 16, 24, 32, 48, 64};
    float tn = 1e30f, tf = 1e30f;
    for (int t : threads)
        for (int b : per_cu) {
            a.near_threads = t;
            a.near_grid = grid_for(c, b);
            const float ms = timed([&] { launch_near(s, a, 3u); });
            if (ms < tn) {
                tn = ms;
                best.near_threads = t;
                best.near_blocks_per_cu = b;
            }
            a.far_threads = t;
            a.far_grid = grid_for(c, b);
            const float mf = timed([&] { launch_far_targets(s, a); });
            if (mf < tf) {
                tf = mf;
                best.far_threads = t;
                best.far_blocks_per_cu = b;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    st = check_launch(c, "autotune");
    if (st != STC_OK) return st;
    if (!ok) return fail(c, STC_ERR_DEVICE, "event timing failed");
    c->shapes[size_class(c->n)] = best;
    *out = best;
    return STC_OK;
}

stc_status stc_set_model(stc_ctx* c, const uint16_t* d_params) {
    if (!c) return STC_ERR_INVALID_ARG;
    if (!c->learned) return fail(c, STC_ERR_STATE, "the context was created without STC_FLAG_LEARNED");
    if (d_params && (reinterpret_cast<uintptr_t>(d_params) & 15u))
        return fail(c, STC_ERR_INVALID_ARG, "d_params must be 16-byte aligned");
    c->model = d_params;
    return STC_OK;
}

stc_status stc_copy_candidates(stc_ctx* c, int64_t cap, int64_t* h_pairs, float* h_out, uint16_t* h_feat,
                               int64_t* n_out) {
    stc_status st = check_ready(c, false);
    if (st != STC_OK) return st;
    if (!c->learned) return fail(c, STC_ERR_STATE, "the context was created without STC_FLAG_LEARNED");
    if (!n_out || cap < 0) return fail(c, STC_ERR_INVALID_ARG, "bad buffer");
    st = stc_sync(c);
    if (st != STC_OK) return st;
    u32 nc = 0;
    if (hipMemcpy(&nc, c->counters + C_CAND, sizeof(u32), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, STC_ERR_DEVICE, "reading counters failed");
    nc = std::min(nc, c->cap);
    *n_out = nc;
    const i64 m = std::min<i64>(nc, cap);
    if (m > 0) {
        std::vector<u64> buf(m);
        if (h_pairs) {
            if (hipMemcpy(buf.data(), c->cand_view ? c->cand_view : c->cand, m * sizeof(u64), hipMemcpyDeviceToHost) !=
                hipSuccess)
                return fail(c, STC_ERR_DEVICE, "copy failed");
            for (i64 i = 0; i < m; ++i) {
                h_pairs[2 * i] = (int64_t)(buf[i] >> 32);
                h_pairs[2 * i + 1] = (int64_t)(buf[i] & 0xffffffffu);
            }
        }
        if (h_out && c->model &&
            hipMemcpy(h_out, c->mlp_out, m * 4 * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
            return fail(c, STC_ERR_DEVICE, "copy failed");
        if (h_feat &&
            hipMemcpy(h_feat, c->feat, m * 16 * sizeof(uint16_t), hipMemcpyDeviceToHost) != hipSuccess)
            return fail(c, STC_ERR_DEVICE, "copy failed");
    }
    return (h_pairs || h_out || h_feat) && nc > cap ? fail(c, STC_ERR_CAPACITY, "buffers too small") : STC_OK;
}

stc_status stc_learned_samples(stc_ctx* c, double abs_tol, int64_t cap, uint16_t* d_features, float* d_labels,
                               double* d_errors, int64_t* n_out) {
    stc_status st = check_ready(c, false);
    if (st != STC_OK) return st;
    if (!c->learned) return fail(c, STC_ERR_STATE, "the context was created without STC_FLAG_LEARNED");
    if (!c->have_upward) return fail(c, STC_ERR_STATE, "call stc_upward first");
    if (!n_out || cap < 0 || !(abs_tol > 0.0) || (cap > 0 && (!d_features || !d_labels || !d_errors)))
        return fail(c, STC_ERR_INVALID_ARG, "bad tolerance or buffers");
    if ((reinterpret_cast<uintptr_t>(d_labels) & 15u) || (reinterpret_cast<uintptr_t>(d_errors) & 7u))
        return fail(c, STC_ERR_INVALID_ARG, "misaligned buffers");
    hipStream_t s = c->stream;
    // candidates of the wider criterion, their features and measured errors
    const TravArgs tc = trav_args(c, c->p.theta_max, 0);
    launch_fill_u32(s, c->sort_zero, kSortZeroWords, 0u);
    launch_traverse_init(s, tc);
    launch_traverse_levels(s, tc, C_FRONT, true, c->cand);
    // samples in (t, s) order, so that training data do not depend on the
    // order in which the traversal appended them (the frontier is free now)
    u64* sorted = nullptr;
    radix_sort(s, c->cand, c->front1, c->counters + C_CAND, c->cap, 0, 32 + c->W,
               sort_scratch(c), &sorted);
    LearnedArgs la = learned_args(c);
    la.cand = sorted;
    c->cand_view = sorted;
    launch_features(s, la);
    EvalArgs a = eval_args(c);
    const u32 lim = (u32)std::min<i64>(cap, 0x7fffffffLL);
    launch_pair_errors(s, la, a, c->p.denominator == STC_DEN_DIST2 ? 1 : 0, lim, d_errors);
    launch_labels(s, la, lim, d_errors, abs_tol, d_labels);
    c->have_lists = false;  // the lists hold only the candidate pass now
    st = check_launch(c, "learned_samples");
    if (st != STC_OK) return st;
    st = stc_sync(c);
    if (st != STC_OK) return st;
    u32 nc = 0;
    if (hipMemcpy(&nc, c->counters + C_CAND, sizeof(u32), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, STC_ERR_DEVICE, "reading counters failed");
    nc = std::min(nc, c->cap);
    *n_out = nc;
    const i64 m = std::min<i64>(nc, cap);
    if (m > 0) {
        const bool ok =
            hipMemcpyAsync(d_features, c->feat, m * 16 * sizeof(uint16_t), hipMemcpyDeviceToDevice, s) == hipSuccess;
        if (!ok || hipStreamSynchronize(s) != hipSuccess) return fail(c, STC_ERR_DEVICE, "copying samples failed");
    }
    return nc > cap && cap > 0 ? fail(c, STC_ERR_CAPACITY, "sample buffers too small") : STC_OK;
}

// --- the network (context-free) ----------------------------------------------

int32_t stc_mlp_param_count(void) { return mlp_param_count(); }

int64_t stc_mlp_workspace_bytes(int64_t n_batch) {
    if (n_batch < 0) return 0;
    return (int64_t)mlp_workspace_floats(n_batch) * (int64_t)sizeof(float);
}

int64_t stc_mlp_calibrate_workspace_bytes(int64_t n) { return n < 0 ? 0 : (int64_t)calib_workspace_bytes(n); }

stc_status stc_mlp_calibrate(void* hip_stream, int64_t n, const uint16_t* d_x, const float* d_y,
                             const uint16_t* d_params, double max_false_accept, double max_under_class, void* d_ws,
                             int64_t ws_bytes, uint16_t* d_params_out, double* d_shifts) {
    if (n < 0 || n > 0x7fffffffLL || !d_params || !d_params_out || !d_shifts || !d_ws) return STC_ERR_INVALID_ARG;
    if (n > 0 && (!d_x || !d_y)) return STC_ERR_INVALID_ARG;
    if (!(max_false_accept >= 0.0 && max_false_accept <= 1.0) || !(max_under_class >= 0.0 && max_under_class <= 1.0))
        return STC_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(d_x) & 15u) || (reinterpret_cast<uintptr_t>(d_y) & 15u) ||
        (reinterpret_cast<uintptr_t>(d_ws) & 15u) || !aligned8(d_shifts))
        return STC_ERR_INVALID_ARG;
    if (ws_bytes < stc_mlp_calibrate_workspace_bytes(n)) return STC_ERR_WORKSPACE;
    launch_mlp_calibrate(static_cast<hipStream_t>(hip_stream), d_x, d_y, n, d_params, max_false_accept,
                         max_under_class, d_ws, d_params_out, d_shifts);
    return hipGetLastError() == hipSuccess ? STC_OK : STC_ERR_DEVICE;
}

stc_status stc_label_scale(void* hip_stream, int64_t n, const double* d_u, double* d_scale) {
    if (n < 0 || !d_scale || !aligned8(d_scale) || (n > 0 && (!d_u || !aligned8(d_u)))) return STC_ERR_INVALID_ARG;
    launch_label_scale(static_cast<hipStream_t>(hip_stream), d_u, n, d_scale);
    return hipGetLastError() == hipSuccess ? STC_OK : STC_ERR_DEVICE;
}

stc_status stc_mlp_forward(void* hip_stream, int64_t n, const uint16_t* d_x, const uint16_t* d_params, float* d_out) {
    if (n < 0 || (n > 0 && (!d_x || !d_params || !d_out))) return STC_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(d_x) & 15u) || (reinterpret_cast<uintptr_t>(d_out) & 15u)) return STC_ERR_INVALID_ARG;
    if (n == 0) return STC_OK;
    launch_mlp_forward(static_cast<hipStream_t>(hip_stream), d_x, n, nullptr, 0, d_params, d_out);
    return hipGetLastError() == hipSuccess ? STC_OK : STC_ERR_DEVICE;
}

stc_status stc_mlp_grad(void* hip_stream, int64_t n, const int32_t* d_index, const uint16_t* d_x, const float* d_y,
                        const uint16_t* d_params, float* d_ws, int64_t ws_bytes, float* d_grad, float* d_loss) {
    if (n < 1 || n > 0x7fffffffLL || !d_x || !d_y || !d_params || !d_ws || !d_grad) return STC_ERR_INVALID_ARG;
    if (ws_bytes < stc_mlp_workspace_bytes(n)) return STC_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(d_x) & 15u) || (reinterpret_cast<uintptr_t>(d_y) & 15u)) return STC_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int nw = launch_mlp_grad(s, d_x, d_y, d_index, n, d_params, d_ws);
    launch_mlp_reduce_adam(s, d_ws, nw, d_grad, d_loss, nullptr, nullptr, nullptr, nullptr, 0.f, 0.9f, 0.999f, 1e-8f, 1);
    return hipGetLastError() == hipSuccess ? STC_OK : STC_ERR_DEVICE;
}

stc_status stc_mlp_train(void* hip_stream, int64_t n_samples, const uint16_t* d_x, const float* d_y, int32_t epochs,
                         int32_t batch, float lr, uint64_t seed, float* d_master, float* d_m1, float* d_m2,
                         uint16_t* d_params, int32_t* d_index, float* d_ws, int64_t ws_bytes, float* d_loss) {
    if (n_samples < 1 || n_samples > 0x7fffffffLL || epochs < 0 || batch < 1 || !(lr > 0.f) || !d_x || !d_y ||
        !d_master || !d_m1 || !d_m2 || !d_params || !d_index || !d_ws)
        return STC_ERR_INVALID_ARG;
    const i64 nb = std::min<i64>(batch, n_samples);
    if (ws_bytes < stc_mlp_workspace_bytes(nb)) return STC_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(d_x) & 15u) || (reinterpret_cast<uintptr_t>(d_y) & 15u)) return STC_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const i64 steps = (n_samples + nb - 1) / nb;
    u64 state = seed * 0x9e3779b97f4a7c15ull + 1;
    auto next = [&state]() {  // splitmix64
        u64 z = (state += 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return z ^ (z >> 31);
    };
    const u64 n = (u64)n_samples;
    launch_mlp_round(s, d_master, d_params);  // the BF16 copy the first step reads
    int step = 0;
    for (int e = 0; e < epochs; ++e) {
        // a bijection i -> (a i + c) mod n with gcd(a, n) = 1
        u64 a = next() % n;
        auto gcd = [](u64 x, u64 y) {
            while (y) {
                const u64 t = x % y;
                x = y;
                y = t;
            }
            return x;
        };
        while (a == 0 || gcd(a, n) != 1) a = (a + 1) % n;
        const u64 cc = next() % n;
        for (i64 b = 0; b < steps; ++b) {
            const i64 base = b * nb;
            const i64 m = std::min<i64>(nb, n_samples - base);
            launch_mlp_batch_index(s, n_samples, base, m, n == 1 ? 1 : a, cc, d_index);
            const int nw = launch_mlp_grad(s, d_x, d_y, d_index, m, d_params, d_ws);
            ++step;
            launch_mlp_reduce_adam(s, d_ws, nw, nullptr, d_loss ? d_loss + (step - 1) : nullptr, d_master, d_m1, d_m2,
                                   d_params, lr, 0.9f, 0.999f, 1e-8f, step);
        }
    }
    return hipGetLastError() == hipSuccess ? STC_OK : STC_ERR_DEVICE;
}

stc_status stc_sync(stc_ctx* c) {
    if (!c) return STC_ERR_INVALID_ARG;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, STC_ERR_DEVICE, "stream synchronisation failed");
    u32 h[C_COUNT];
    u32 f[F_COUNT];
    if (hipMemcpy(h, c->counters, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(f, c->flags, sizeof(f), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, STC_ERR_DEVICE, "reading device flags failed");
    if (h[C_OVERFLOW] || h[C_TLIST] > c->cap || h[C_NLIST] > c->cap)
        return fail(c, STC_ERR_CAPACITY, "interaction list or frontier exceeded list_capacity");
    if (f[F_SLOTS]) return fail(c, STC_ERR_CAPACITY, "proxy storage slots exceeded");
    if (f[F_NONFINITE]) return fail(c, STC_ERR_NONFINITE, "non-finite particle position");
    if (f[F_NONFINITE_CHARGE]) return fail(c, STC_ERR_NONFINITE, "non-finite vorticity or area (charge zeta A)");
    if (f[F_SORT_SPIN]) return fail(c, STC_ERR_DEVICE, "a sort's look-back exceeded its spin bound");
    return STC_OK;
}

stc_status stc_list_counts(stc_ctx* c, int64_t counts[4], int64_t kernel_evals[4]) {
    stc_status st = check_ready(c, true);
    if (st != STC_OK) return st;
    st = stc_sync(c);
    if (st != STC_OK) return st;
    unsigned long long h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    (void)hipMemsetAsync(c->evals, 0, sizeof(h), c->stream);
    launch_count_evals(c->stream, c->tlist, c->counters + C_TLIST, c->cap, c->W, c->DB, c->cls, c->nbeg, c->nend, 0,
                       c->evals);
    launch_count_evals(c->stream, c->nlist, c->counters + C_NLIST, c->cap, c->W, c->DB, c->cls, c->nbeg, c->nend, 1,
                       c->evals + 4);
    if (hipStreamSynchronize(c->stream) != hipSuccess ||
        hipMemcpy(h, c->evals, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, STC_ERR_DEVICE, "counting list work failed");
    if (counts) {
        counts[0] = (int64_t)h[2];
        counts[1] = (int64_t)h[3];
        counts[2] = (int64_t)h[6];
        counts[3] = (int64_t)h[7];
    }
    if (kernel_evals) {
        kernel_evals[0] = (int64_t)h[0];
        kernel_evals[1] = (int64_t)h[1];
        kernel_evals[2] = (int64_t)h[4];
        kernel_evals[3] = (int64_t)h[5];
    }
    return STC_OK;
}

static stc_status copy_list_impl(stc_ctx* c, int32_t type, int64_t cap, int64_t* h_pairs, int32_t* h_class,
                                 int64_t* n_out) {
    stc_status st = check_ready(c, true);
    if (st != STC_OK) return st;
    if (type < 0 || type > 3 || cap < 0 || (cap > 0 && !h_pairs && !h_class) || !n_out)
        return fail(c, STC_ERR_INVALID_ARG, "bad list type or buffer");
    st = stc_sync(c);
    if (st != STC_OK) return st;
    u32 cnt[2];
    if (hipMemcpy(cnt, c->counters, sizeof(cnt), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, STC_ERR_DEVICE, "reading counters failed");
    const bool tl = type <= 1;
    const u32 len = std::min(tl ? cnt[0] : cnt[1], c->cap);
    std::vector<u64> buf(len);
    if (len && hipMemcpy(buf.data(), tl ? c->tlist : c->nlist, len * sizeof(u64), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, STC_ERR_DEVICE, "copying list failed");
    const u64 mask = ((u64)1 << c->W) - 1;
    const u64 want = (u64)(type & 1);
    int64_t k = 0;
    for (u32 i = 0; i < len; ++i) {
        const u64 key = buf[i];
        if (((key >> c->W) & 1u) != want) continue;
        if (k < cap) {
            if (h_pairs) {
                h_pairs[2 * k] = (int64_t)(key >> (c->W + 1 + c->DB));
                h_pairs[2 * k + 1] = (int64_t)(key & mask);
            }
            if (h_class) h_class[k] = (int32_t)((key >> (c->W + 1)) & ((1u << c->DB) - 1u));
        }
        ++k;
    }
    *n_out = k;
    if (h_pairs == nullptr && h_class == nullptr) return STC_OK;  // size query
    return k > cap ? fail(c, STC_ERR_CAPACITY, "output buffer too small") : STC_OK;
}

stc_status stc_copy_list(stc_ctx* c, int32_t type, int64_t cap, int64_t* h_pairs, int64_t* n_out) {
    return copy_list_impl(c, type, cap, h_pairs, nullptr, n_out);
}

stc_status stc_copy_list_classes(stc_ctx* c, int32_t type, int64_t cap, int32_t* h_class, int64_t* n_out) {
    return copy_list_impl(c, type, cap, nullptr, h_class, n_out);
}

stc_status stc_copy_tree(stc_ctx* c, int64_t n, int32_t* h_perm, int64_t node_cap, int32_t* h_count) {
    stc_status st = check_ready(c, false);
    if (st != STC_OK) return st;
    if (h_perm && n != c->n) return fail(c, STC_ERR_INVALID_ARG, "n differs from the built tree");
    if (h_count && node_cap < c->n_nodes) return fail(c, STC_ERR_INVALID_ARG, "node_cap too small");
    const i64 un = c->used_nodes;
    st = stc_sync(c);
    if (st != STC_OK) return st;
    if (h_perm && n > 0 && hipMemcpy(h_perm, c->perm, n * sizeof(i32), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, STC_ERR_DEVICE, "copying perm failed");
    if (h_count) {
        std::vector<i32> b(un), e(un);
        if (hipMemcpy(b.data(), c->nbeg, un * sizeof(i32), hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(e.data(), c->nend, un * sizeof(i32), hipMemcpyDeviceToHost) != hipSuccess)
            return fail(c, STC_ERR_DEVICE, "copying node ranges failed");
        for (i64 i = 0; i < c->n_nodes; ++i) h_count[i] = i < un ? e[i] - b[i] : 0;
    }
    return STC_OK;
}

stc_status stc_copy_proxy_charges(stc_ctx* c, int64_t node_id, double* h_w) {
    stc_status st = check_ready(c, false);
    if (st != STC_OK) return st;
    if (!c->have_upward) return fail(c, STC_ERR_STATE, "call stc_upward first");
    if (node_id < 0 || node_id >= c->used_nodes || !h_w) return fail(c, STC_ERR_INVALID_ARG, "bad node id or buffer");
    st = stc_sync(c);
    if (st != STC_OK) return st;
    i32 b = 0, e = 0;
    if (hipMemcpy(&b, c->nbeg + node_id, sizeof(i32), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(&e, c->nend + node_id, sizeof(i32), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, STC_ERR_DEVICE, "copy failed");
    if (e - b <= c->p.n_crit) {
        for (int m = 0; m < c->np; ++m) h_w[m] = 0.0;
        return STC_OK;
    }
    i32 sl = -1;
    if (hipMemcpy(&sl, c->slot + node_id, sizeof(i32), hipMemcpyDeviceToHost) != hipSuccess || sl < 0)
        return fail(c, STC_ERR_DEVICE, "copy failed");
    std::vector<Prox> pr(c->np);
    const size_t rec = (size_t)sl * c->NPT + c->cls.poff[c->fb_class];
    if (hipMemcpy(pr.data(), c->prox + rec, c->np * sizeof(Prox), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, STC_ERR_DEVICE, "copy failed");
    for (int m = 0; m < c->np; ++m) h_w[m] = pr[m].w;
    return STC_OK;
}

stc_status stc_node_geometry(const stc_ctx* c, int64_t node_id, double* h_v9, double* h_c3, double* h_r) {
    if (!c || node_id < 0 || node_id >= c->n_nodes) return STC_ERR_INVALID_ARG;
    const i64 local = node_id & (((i64)1 << c->NB) - 1);
    if (local >= c->n_local) return STC_ERR_INVALID_ARG;
    const NodeGeo& g = c->geo_host[local];
    if (h_v9)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) h_v9[3 * a + b] = g.v[a][b];
    if (h_c3)
        for (int b = 0; b < 3; ++b) h_c3[b] = g.c[b];
    if (h_r) *h_r = g.r;
    return STC_OK;
}

stc_status stc_geometry_tables(int32_t max_level, double* h_v, double* h_c, double* h_r) {
    if (max_level < 0 || max_level > 12) return STC_ERR_INVALID_ARG;
    std::vector<NodeGeo> geo;
    try {
        build_tree_geometry(max_level, geo);
    } catch (...) {
        return STC_ERR_ALLOC;
    }
    for (size_t i = 0; i < geo.size(); ++i) {
        if (h_v)
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) h_v[9 * i + 3 * a + b] = geo[i].v[a][b];
        if (h_c)
            for (int b = 0; b < 3; ++b) h_c[3 * i + b] = geo[i].c[b];
        if (h_r) h_r[i] = geo[i].r;
    }
    return STC_OK;
}

stc_status stc_reference_tables(int32_t degree, double* h_points, double* h_vinv) {
    RefTables t;
    if (!build_reference_tables(degree, t) || degree > kMaxDegree) return STC_ERR_INVALID_ARG;
    if (h_points) std::memcpy(h_points, t.points.data(), t.points.size() * sizeof(double));
    if (h_vinv) std::memcpy(h_vinv, t.vinv.data(), t.vinv.size() * sizeof(double));
    return STC_OK;
}

stc_status stc_set_timing(stc_ctx* c, int32_t max_evals) { return stc_set_timing_phases(c, max_evals, 0x3f); }

stc_status stc_set_timing_phases(stc_ctx* c, int32_t max_evals, uint32_t phase_mask) {
    if (!c || max_evals < 0 || max_evals > 100000 || (phase_mask & ~0x3fu)) return STC_ERR_INVALID_ARG;
    c->t_mask = phase_mask;
    (void)hipStreamSynchronize(c->stream);
    for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
    c->tev.clear();
    c->t_max = c->t_used = 0;
    if (max_evals == 0) return STC_OK;
    c->tev.resize((size_t)max_evals * 12);
    for (auto& e : c->tev)
        if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
            return fail(c, STC_ERR_DEVICE, "hipEventCreate failed");
        }
    c->t_max = max_evals;
    return STC_OK;
}

stc_status stc_phase_times(stc_ctx* c, double ms[6], int64_t* n_evals) {
    if (!c || !ms || !n_evals) return STC_ERR_INVALID_ARG;
    for (int p = 0; p < 6; ++p) ms[p] = 0.0;
    *n_evals = 0;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, STC_ERR_DEVICE, "synchronisation failed");
    for (int k = 0; k < c->t_used; ++k) {
        for (int p = 0; p < 6; ++p) {
            if (!((c->t_mask >> p) & 1u)) continue;
            float t = 0.f;
            if (hipEventElapsedTime(&t, c->tev[(size_t)k * 12 + 2 * p], c->tev[(size_t)k * 12 + 2 * p + 1]) != hipSuccess)
                return fail(c, STC_ERR_DEVICE, "event timing failed (was every phase of the evaluation run?)");
            ms[p] += t;
        }
    }
    *n_evals = c->t_used;
    c->t_used = 0;
    return STC_OK;
}

// --- one evaluation captured in a HIP graph ------------------------------------

struct stc_graph {
    stc_ctx* ctx = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};  // around the last replay, on the launch stream
    bool launched = false;
};

stc_status stc_velocity_graph(stc_ctx* c, int64_t n, const double* d_x, const double* d_zeta, const double* d_area,
                              double* d_u, stc_graph** out) {
    if (!c || !out) return STC_ERR_INVALID_ARG;
    *out = nullptr;
    if (n < 1 || n > c->n_max) return fail(c, STC_ERR_INVALID_ARG, "n out of range [1, n_max]");
    if (!d_x || !d_zeta || !d_area || !d_u || !aligned8(d_x) || !aligned8(d_zeta) || !aligned8(d_area) ||
        !aligned8(d_u))
        return fail(c, STC_ERR_INVALID_ARG, "NULL or misaligned pointer");
    stc_graph* g = new (std::nothrow) stc_graph();
    if (!g) return STC_ERR_ALLOC;
    g->ctx = c;
    for (hipEvent_t& e : g->ev)
        if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
            stc_graph_destroy(g);
            return fail(c, STC_ERR_DEVICE, "hipEventCreate failed");
        }
    if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        stc_graph_destroy(g);
        return fail(c, STC_ERR_DEVICE, "creating the capture stream failed");
    }
    // capture on the context's capture stream, with the context's phase
    // timing off (its events belong to eager evaluations)
    const int tmax = c->t_max;
    c->t_max = 0;
    hipStream_t user = c->stream;
    c->stream = c->cap_stream;
    hipGraph_t graph = nullptr;
    stc_status st = STC_OK;
    if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        st = fail(c, STC_ERR_DEVICE, "hipStreamBeginCapture failed");
    } else {
        const i64 off[2] = {0, n};
        st = do_build(c, 1, off, d_x);
        if (st == STC_OK) st = do_upward_traverse(c, d_zeta, d_area);
        if (st == STC_OK) st = do_eval(c, true, true, d_u, false);
        const hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
        if (st == STC_OK && e != hipSuccess) st = fail(c, STC_ERR_DEVICE, "hipStreamEndCapture failed");
    }
    c->stream = user;
    c->t_max = tmax;
    if (st == STC_OK && hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        g->exec = nullptr;
        st = fail(c, STC_ERR_DEVICE, "hipGraphInstantiate failed");
    }
    if (graph) (void)hipGraphDestroy(graph);
    if (st != STC_OK) {
        stc_graph_destroy(g);
        return st;
    }
    *out = g;
    return STC_OK;
}

stc_status stc_graph_launch(stc_graph* g) {
    if (!g || !g->exec) return STC_ERR_INVALID_ARG;
    hipStream_t s = g->ctx->stream;
    if (hipEventRecord(g->ev[0], s) != hipSuccess || hipGraphLaunch(g->exec, s) != hipSuccess ||
        hipEventRecord(g->ev[1], s) != hipSuccess)
        return fail(g->ctx, STC_ERR_DEVICE, "hipGraphLaunch failed");
    g->launched = true;
    return STC_OK;
}

stc_status stc_graph_last_ms(stc_graph* g, double* ms) {
    if (!g || !ms) return STC_ERR_INVALID_ARG;
    *ms = 0.0;
    if (!g->launched) return fail(g->ctx, STC_ERR_STATE, "the graph has not been launched");
    if (hipEventSynchronize(g->ev[1]) != hipSuccess) return fail(g->ctx, STC_ERR_DEVICE, "synchronisation failed");
    float t = 0.f;
    if (hipEventElapsedTime(&t, g->ev[0], g->ev[1]) != hipSuccess)
        return fail(g->ctx, STC_ERR_DEVICE, "event timing failed");
    *ms = t;
    return STC_OK;
}

stc_status stc_graph_destroy(stc_graph* g) {
    if (!g) return STC_ERR_INVALID_ARG;
    if (g->ctx) (void)hipStreamSynchronize(g->ctx->stream);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    for (hipEvent_t e : g->ev)
        if (e) (void)hipEventDestroy(e);
    delete g;
    return STC_OK;
}

const char* stc_last_error(const stc_ctx* c) { return c ? c->err.c_str() : ""; }

}  // extern "C"
