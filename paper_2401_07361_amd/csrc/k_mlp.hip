// The learned form's network: a multilayer perceptron 12 -> 64 -> 64 -> 4
// with ReLU hidden layers, BF16 weights and activations and FP32
// accumulation on the matrix cores (v_mfma_f32_16x16x16_bf16), forward and
// backward.
//
// Parameters, one flat vector of 5252 values (row-major blocks):
//   W1 [12][64] (input feature f -> hidden h), b1 [64], W2 [64][64],
//   b2 [64], W3 [64][4], b3 [4].
// Inputs are rows of 16 BF16 values (features 12..15 are zero).  Outputs:
//   o0 = acceptance logit, o1..o3 = ordinal logits (degree above 4, 6, 8).
//
// The layers run transposed, Z^T = W^T X^T: hidden units are the MFMA rows,
// 16 samples its columns.  The 16x16 result tile of one layer then sits in
// the registers exactly as the B operand of the next layer expects (lane l
// holds rows 4(l/16)..4(l/16)+3 of column l%16), so activations never leave
// registers in the forward pass.  Weight gradients contract over samples;
// their operands are staged through LDS in [unit][sample] order.
//
// Loss (per sample, mean over the batch): a(y0) BCE(o0, y0) + y0 * sum_k
// h(y_k) BCE(o_k, y_k), k = 1..3 -- the ordinal targets count only for
// accepted samples; the costly mistakes weigh more: a sample labelled reject
// kWReject times in the acceptance term, a "degree above" target kWHigher
// times in its ordinal term (the network's own decisions then lean to the
// safe side, and the calibration after training moves the biases less).
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "kernels.hpp"

namespace stc {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int P_W1 = 0, P_B1 = 768, P_W2 = 832, P_B2 = 4928, P_W3 = 4992, P_B3 = 5248, P_N = 5252;
constexpr int WS_STRIDE = P_N + 1;  // per-wave partial gradients + loss

__device__ __forceinline__ float bf2f(u16 h) { return __uint_as_float((u32)h << 16); }

// round to nearest even
__device__ __forceinline__ u16 f2bf(float f) {
    u32 u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x4 pack4(u16 a, u16 b, u16 c, u16 d) {
    bf16x4 v;
    v[0] = (short)a;
    v[1] = (short)b;
    v[2] = (short)c;
    v[3] = (short)d;
    return v;
}

__device__ __forceinline__ bf16x4 to_bf16x4(f32x4 f) { return pack4(f2bf(f[0]), f2bf(f[1]), f2bf(f[2]), f2bf(f[3])); }

// parameters in LDS (BF16 weights, FP32 biases)
struct ParamShared {
    u16 w[P_N];
    float b1[64], b2[64], b3[4];
};

__device__ void load_params(const u16* __restrict__ P, ParamShared& ps) {
    for (int i = threadIdx.x; i < P_N; i += blockDim.x) ps.w[i] = P[i];
    for (int i = threadIdx.x; i < 64; i += blockDim.x) {
        ps.b1[i] = bf2f(P[P_B1 + i]);
        ps.b2[i] = bf2f(P[P_B2 + i]);
    }
    if (threadIdx.x < 4) ps.b3[threadIdx.x] = bf2f(P[P_B3 + threadIdx.x]);
    __syncthreads();
}

// A fragments of the forward layers for lane (r = l % 16, g = l / 16)
struct FwdFrag {
    bf16x4 a1[4], a2[4][4], a3[4];
};

__device__ void fwd_frags(const ParamShared& ps, int r, int g, FwdFrag& F) {
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        u16 e[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int f = 4 * g + v;
            e[v] = f < 12 ? ps.w[P_W1 + f * 64 + 16 * mt + r] : (u16)0;
        }
        F.a1[mt] = pack4(e[0], e[1], e[2], e[3]);
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) {
#pragma unroll
            for (int v = 0; v < 4; ++v) e[v] = ps.w[P_W2 + (16 * kt + 4 * g + v) * 64 + 16 * mt + r];
            F.a2[mt][kt] = pack4(e[0], e[1], e[2], e[3]);
        }
    }
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) {
        u16 e[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) e[v] = r < 4 ? ps.w[P_W3 + (16 * kt + 4 * g + v) * 4 + r] : (u16)0;
        F.a3[kt] = pack4(e[0], e[1], e[2], e[3]);
    }
}

// Forward pass of one tile of 16 samples (x: this lane's B fragment, i.e.
// features 4g..4g+3 of sample r).  Returns pre-activations (bias added) of
// both hidden layers, their BF16 activations and the output tile (bias
// added; rows 0..3 = outputs, valid in lanes with g == 0).
__device__ __forceinline__ void forward_tile(const FwdFrag& F, const ParamShared& ps, int g, bf16x4 x,
                                             f32x4 z1[4], bf16x4 h1[4], f32x4 z2[4], bf16x4 h2[4], f32x4& z3) {
    const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        f32x4 z = mfma16(F.a1[mt], x, zero);
        f32x4 h;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            z[v] += ps.b1[16 * mt + 4 * g + v];
            h[v] = z[v] > 0.f ? z[v] : 0.f;
        }
        z1[mt] = z;
        h1[mt] = to_bf16x4(h);
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        f32x4 z = zero;
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) z = mfma16(F.a2[mt][kt], h1[kt], z);
        f32x4 h;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            z[v] += ps.b2[16 * mt + 4 * g + v];
            h[v] = z[v] > 0.f ? z[v] : 0.f;
        }
        z2[mt] = z;
        h2[mt] = to_bf16x4(h);
    }
    f32x4 z = zero;
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) z = mfma16(F.a3[kt], h2[kt], z);
#pragma unroll
    for (int v = 0; v < 4; ++v) z[v] += (g == 0) ? ps.b3[v] : 0.f;
    z3 = z;
}

__device__ __forceinline__ bf16x4 load_x(const u16* __restrict__ X, i64 row, int g, bool ok) {
    if (!ok) return pack4(0, 0, 0, 0);
    const uint2 w = *reinterpret_cast<const uint2*>(X + row * 16 + 4 * g);
    return pack4((u16)(w.x & 0xffffu), (u16)(w.x >> 16), (u16)(w.y & 0xffffu), (u16)(w.y >> 16));
}

// Forward over n rows (n from *d_n when given, clamped to cap): one wave per
// 16-row tile, persistent over tiles.
__global__ __launch_bounds__(256) void k_mlp_forward(const u16* __restrict__ X, i64 n, const u32* __restrict__ d_n,
                                                      u32 cap, const u16* __restrict__ P, float* __restrict__ out) {
    __shared__ ParamShared ps;
    load_params(P, ps);
    if (d_n) {
        const u32 m = *d_n;
        n = m < cap ? m : cap;
    }
    const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
    FwdFrag F;
    fwd_frags(ps, r, g, F);
    const i64 tiles = (n + 15) / 16;
    const i64 wave = (i64)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const i64 nw = (i64)gridDim.x * (blockDim.x / 64);
    for (i64 tile = wave; tile < tiles; tile += nw) {
        const i64 row = tile * 16 + r;
        const bool ok = row < n;
        f32x4 z1[4], z2[4], z3;
        bf16x4 h1[4], h2[4];
        forward_tile(F, ps, g, load_x(X, row, g, ok), z1, h1, z2, h2, z3);
        if (ok && g == 0) *reinterpret_cast<float4*>(out + row * 4) = make_float4(z3[0], z3[1], z3[2], z3[3]);
    }
}

__device__ __forceinline__ float sigmoid(float o) { return 1.f / (1.f + __expf(-o)); }

constexpr float kWReject = 8.f;  // weight of a reject-labelled sample's acceptance term
constexpr float kWHigher = 8.f;  // weight of a "degree above" ordinal target

// BCE with logits: max(o, 0) - o y + log(1 + exp(-|o|))
__device__ __forceinline__ float bce(float o, float y) { return fmaxf(o, 0.f) - o * y + log1pf(__expf(-fabsf(o))); }

// per-wave LDS for the weight-gradient operands, [unit][sample]
struct WaveStage {
    u16 x[16][16];
    u16 h1[64][16];
    u16 dz1[64][16];
    u16 h2[64][16];
    u16 dz2[64][16];
    u16 dz3[16][16];
};

__device__ __forceinline__ bf16x4 lds4(const u16* p) {
    const uint2 w = *reinterpret_cast<const uint2*>(p);
    return pack4((u16)(w.x & 0xffffu), (u16)(w.x >> 16), (u16)(w.y & 0xffffu), (u16)(w.y >> 16));
}

__device__ __forceinline__ void stage_tile(u16 (*dst)[16], int unit0, int g, int r, bf16x4 v) {
#pragma unroll
    for (int k = 0; k < 4; ++k) dst[unit0 + 4 * g + k][r] = (u16)v[k];
}

// sum over the 16 lanes that share g (the 16 samples of a tile row)
__device__ __forceinline__ float sum16(float v) {
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Gradient of the mean loss over rows idx[0..nb) (idx NULL: rows 0..nb).
// Each wave writes its partial gradient (and loss) to ws[wave]; a block's
// waves take tiles in lockstep so that the block barriers are uniform.
__global__ __launch_bounds__(256) void k_mlp_grad(const u16* __restrict__ X, const float* __restrict__ Y,
                                                   const i32* __restrict__ idx, i64 nb, const u16* __restrict__ P,
                                                   float* __restrict__ ws) {
    __shared__ ParamShared ps;
    __shared__ WaveStage st[4];
    load_params(P, ps);
    const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4, w = threadIdx.x >> 6;
    FwdFrag F;
    fwd_frags(ps, r, g, F);
    // backward A fragments: W3 (dH2^T = W3 dZ3^T) and W2 (dH1^T = W2 dZ2^T)
    bf16x4 c3[4], c2[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        u16 e[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) e[v] = (g == 0) ? ps.w[P_W3 + (16 * mt + r) * 4 + v] : (u16)0;
        c3[mt] = pack4(e[0], e[1], e[2], e[3]);
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) {
#pragma unroll
            for (int v = 0; v < 4; ++v) e[v] = ps.w[P_W2 + (16 * mt + r) * 64 + 16 * kt + 4 * g + v];
            c2[mt][kt] = pack4(e[0], e[1], e[2], e[3]);
        }
    }
    const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
    f32x4 gW1[4], gW2[4][4], gW3[4], gb1[4], gb2[4], gb3 = zero;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        gW1[i] = gW3[i] = gb1[i] = gb2[i] = zero;
#pragma unroll
        for (int j = 0; j < 4; ++j) gW2[i][j] = zero;
    }
    float loss = 0.f;
    const float inv_b = nb > 0 ? 1.f / (float)nb : 0.f;
    const i64 tiles = (nb + 15) / 16;
    const int wpb = blockDim.x / 64;
    WaveStage& S = st[w];
    for (i64 t0 = (i64)blockIdx.x * wpb; t0 < tiles; t0 += (i64)gridDim.x * wpb) {
        const i64 tile = t0 + w;
        const i64 j = tile * 16 + r;
        const bool ok = tile < tiles && j < nb;
        const i64 row = ok ? (idx ? (i64)idx[j] : j) : 0;
        const bf16x4 x = load_x(X, row, g, ok);
        f32x4 z1[4], z2[4], z3;
        bf16x4 h1[4], h2[4];
        forward_tile(F, ps, g, x, z1, h1, z2, h2, z3);
        // output gradient (rows 0..3 = outputs, lanes g == 0)
        f32x4 d3 = zero;
        if (ok && g == 0) {
            const float4 y = *reinterpret_cast<const float4*>(Y + row * 4);
            const float yv[4] = {y.x, y.y, y.z, y.w};
            const float wa = 1.f + (kWReject - 1.f) * (1.f - yv[0]);
            loss += wa * bce(z3[0], yv[0]);
            d3[0] = wa * (sigmoid(z3[0]) - yv[0]) * inv_b;
#pragma unroll
            for (int k = 1; k < 4; ++k) {
                const float wo = 1.f + (kWHigher - 1.f) * yv[k];
                loss += yv[0] * wo * bce(z3[k], yv[k]);
                d3[k] = yv[0] * wo * (sigmoid(z3[k]) - yv[k]) * inv_b;
            }
        }
        gb3 += d3;
        const bf16x4 d3b = to_bf16x4(d3);
        // dZ2^T = (W3 dZ3^T) * relu'(Z2^T)
        bf16x4 d2b[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            f32x4 d = mfma16(c3[mt], d3b, zero);
#pragma unroll
            for (int v = 0; v < 4; ++v) d[v] = z2[mt][v] > 0.f ? d[v] : 0.f;
            gb2[mt] += d;
            d2b[mt] = to_bf16x4(d);
        }
        // dZ1^T = (W2 dZ2^T) * relu'(Z1^T)
        bf16x4 d1b[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            f32x4 d = zero;
#pragma unroll
            for (int kt = 0; kt < 4; ++kt) d = mfma16(c2[mt][kt], d2b[kt], d);
#pragma unroll
            for (int v = 0; v < 4; ++v) d[v] = z1[mt][v] > 0.f ? d[v] : 0.f;
            gb1[mt] += d;
            d1b[mt] = to_bf16x4(d);
        }
        // stage [unit][sample] operands for the weight gradients
        stage_tile(S.x, 0, g, r, x);
        stage_tile(S.dz3, 0, g, r, d3b);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            stage_tile(S.h1, 16 * mt, g, r, h1[mt]);
            stage_tile(S.dz1, 16 * mt, g, r, d1b[mt]);
            stage_tile(S.h2, 16 * mt, g, r, h2[mt]);
            stage_tile(S.dz2, 16 * mt, g, r, d2b[mt]);
        }
        __syncthreads();
        // dW1 = X^T dZ1, dW2 = H1^T dZ2, dW3 = H2^T dZ3 (K = the 16 samples)
        const bf16x4 ax = lds4(&S.x[r][4 * g]);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) gW1[nt] = mfma16(ax, lds4(&S.dz1[16 * nt + r][4 * g]), gW1[nt]);
        const bf16x4 b3 = lds4(&S.dz3[r][4 * g]);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const bf16x4 ah1 = lds4(&S.h1[16 * mt + r][4 * g]);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) gW2[mt][nt] = mfma16(ah1, lds4(&S.dz2[16 * nt + r][4 * g]), gW2[mt][nt]);
            gW3[mt] = mfma16(lds4(&S.h2[16 * mt + r][4 * g]), b3, gW3[mt]);
        }
        __syncthreads();
    }
    // per-wave partials
    float* o = ws + ((i64)blockIdx.x * wpb + w) * WS_STRIDE;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int f = 4 * g + v;
            if (f < 12) o[P_W1 + f * 64 + 16 * nt + r] = gW1[nt][v];
        }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * mt + 4 * g + v;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) o[P_W2 + row * 64 + 16 * nt + r] = gW2[mt][nt][v];
            if (r < 4) o[P_W3 + row * 4 + r] = gW3[mt][v];
            const float s1 = sum16(gb1[mt][v]), s2 = sum16(gb2[mt][v]);
            if (r == 0) {
                o[P_B1 + row] = s1;
                o[P_B2 + row] = s2;
            }
        }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const float s3 = sum16(gb3[v]);
        if (g == 0 && r == 0) o[P_B3 + v] = s3;
    }
    float lsum = loss;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) lsum += __shfl_xor(lsum, off, 64);
    if (lane == 0) o[P_N] = lsum * inv_b;
}

// Sums the per-wave partials in a fixed order (gradient, loss) and, with
// lr > 0, applies one Adam step to the FP32 master weights and writes their
// BF16 copy.
__global__ __launch_bounds__(256) void k_mlp_reduce_adam(const float* __restrict__ ws, int nwaves,
                                                          float* __restrict__ grad, float* __restrict__ loss,
                                                          float* __restrict__ master, float* __restrict__ m1,
                                                          float* __restrict__ m2, u16* __restrict__ P, float lr,
                                                          float beta1, float beta2, float eps, float bc1, float bc2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > P_N) return;
    float s = 0.f;
    for (int w = 0; w < nwaves; ++w) s += ws[(i64)w * WS_STRIDE + p];
    if (p == P_N) {
        if (loss) *loss = s;
        return;
    }
    if (grad) grad[p] = s;
    if (lr > 0.f && master) {
        const float a = beta1 * m1[p] + (1.f - beta1) * s;
        const float b = beta2 * m2[p] + (1.f - beta2) * s * s;
        m1[p] = a;
        m2[p] = b;
        const float th = master[p] - lr * (a / bc1) / (sqrtf(b / bc2) + eps);
        master[p] = th;
        P[p] = f2bf(th);
    }
}

// idx[i] = (a (base + i) + c) mod n: a fixed bijection of [0, n) per epoch
// (gcd(a, n) = 1, a and c reduced mod n < 2^31), walked in batches.
__global__ __launch_bounds__(256) void k_mlp_batch_index(i64 n, i64 base, i64 nb, u64 a, u64 c, i32* __restrict__ idx) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    const u64 k = (u64)((base + i) % n);
    idx[i] = (i32)((a * k + c) % (u64)n);
}

__global__ __launch_bounds__(256) void k_mlp_round(const float* __restrict__ master, u16* __restrict__ P) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < P_N) P[p] = f2bf(master[p]);
}

// --- calibration of the output biases ---------------------------------------
// The network's own decisions are shifted so that on the labelled samples at
// most a given fraction is accepted against its label (b3[0] -= da) and at
// most a given fraction of the correctly accepted ones gets a lower degree
// class than labelled (b3[1..3] += dc), da and dc the smallest values of the
// grid 0, geomspace(1e-3, 64, 200) that meet the bars (the largest if none).
// Each sample maps to the number of grid values below its threshold, so one
// histogram per bar gives the violation count of every grid value.

// # of grid values g[k] (ascending) with g[k] < v (strict) or <= v
__device__ __forceinline__ int grid_rank(const CalibGrid& g, double v, bool inclusive) {
    int lo = 0, hi = CalibGrid::K;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (inclusive ? (g.d[mid] <= v) : (g.d[mid] < v)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// false accepts: a sample labelled "reject" is accepted at shift d iff o0 - d > 0
__global__ __launch_bounds__(256) void k_calib_accept(const float* __restrict__ out, const float* __restrict__ y,
                                                      i64 n, CalibGrid g, u32* __restrict__ hist) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || y[4 * i] > 0.f) return;
    atomicAdd(&hist[grid_rank(g, (double)out[4 * i], false)], 1u);
}

// smallest grid index k whose violation count (samples of rank > k) is at
// most max_rate of the denominator (n, or the count in hist[K + 1]); writes
// the shift to sel[slot] (one thread: K + 1 bins)
__global__ void k_calib_select(const u32* __restrict__ hist, i64 n, double max_rate, CalibGrid g, int slot,
                               double* __restrict__ sel) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double den = n >= 0 ? (double)n : (double)hist[CalibGrid::K + 1];
    if (!(den > 0.0)) {
        sel[slot] = 0.0;
        return;
    }
    u64 above = 0;  // samples of rank > k
    for (int r = 1; r <= CalibGrid::K; ++r) above += hist[r];
    for (int k = 0; k < CalibGrid::K; ++k) {
        if ((double)above / den <= max_rate) {
            sel[slot] = g.d[k];
            return;
        }
        above -= hist[k + 1];
    }
    sel[slot] = g.d[CalibGrid::K - 1];
}

// under-classed: among samples labelled "accept" that the shifted network
// accepts (o0 > da), one needing `need` ordinal steps gets fewer at shift d
// iff fewer than `need` of o1..o3 exceed -d, i.e. iff d <= the need-th
// smallest of -o1..-o3; hist[K + 1] counts the kept samples
__global__ __launch_bounds__(256) void k_calib_class(const float* __restrict__ out, const float* __restrict__ y,
                                                     i64 n, CalibGrid g, const double* __restrict__ sel,
                                                     u32* __restrict__ hist) {
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !(y[4 * i] > 0.f) || !((double)out[4 * i] > sel[0])) return;
    atomicAdd(&hist[CalibGrid::K + 1], 1u);
    const int need = (int)(y[4 * i + 1] + y[4 * i + 2] + y[4 * i + 3] + 0.5f);
    if (need < 1) return;
    double v0 = -(double)out[4 * i + 1], v1 = -(double)out[4 * i + 2], v2 = -(double)out[4 * i + 3];
    if (v0 > v1) { const double t = v0; v0 = v1; v1 = t; }
    if (v1 > v2) { const double t = v1; v1 = v2; v2 = t; }
    if (v0 > v1) { const double t = v0; v0 = v1; v1 = t; }
    const double th = need == 1 ? v0 : (need == 2 ? v1 : v2);
    atomicAdd(&hist[grid_rank(g, th, true)], 1u);
}

// shifted parameters: the FP64 shift applied to the BF16 bias, rounded to
// FP32 and then to BF16 (nearest even both times)
__global__ __launch_bounds__(256) void k_calib_apply(const u16* __restrict__ P, const double* __restrict__ sel,
                                                     u16* __restrict__ Q) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P_N) return;
    u16 v = P[p];
    if (p >= P_B3) {
        const double b = (double)bf2f(v) + (p == P_B3 ? -sel[0] : sel[1]);
        v = f2bf((float)b);
    }
    Q[p] = v;
}

}  // namespace

int mlp_param_count() { return P_N; }

void launch_mlp_round(hipStream_t s, const float* master, u16* P) {
    hipLaunchKernelGGL(k_mlp_round, dim3((P_N + 255) / 256), dim3(256), 0, s, master, P);
}

i64 mlp_workspace_floats(i64 n_batch) {
    const i64 tiles = (n_batch + 15) / 16;
    const i64 blocks = std::min<i64>(std::max<i64>((tiles + 3) / 4, 1), 256);
    return blocks * 4 * WS_STRIDE;
}

void launch_mlp_forward(hipStream_t s, const u16* X, i64 n, const u32* d_n, u32 cap, const u16* P, float* out) {
    const i64 rows = d_n ? (i64)cap : n;
    const i64 tiles = (rows + 15) / 16;
    const unsigned grid = (unsigned)std::min<i64>(std::max<i64>((tiles + 3) / 4, 1), 1024);
    hipLaunchKernelGGL(k_mlp_forward, dim3(grid), dim3(256), 0, s, X, n, d_n, cap, P, out);
}

int launch_mlp_grad(hipStream_t s, const u16* X, const float* Y, const i32* idx, i64 nb, const u16* P, float* ws) {
    const i64 tiles = (nb + 15) / 16;
    const int blocks = (int)std::min<i64>(std::max<i64>((tiles + 3) / 4, 1), 256);
    hipLaunchKernelGGL(k_mlp_grad, dim3(blocks), dim3(256), 0, s, X, Y, idx, nb, P, ws);
    return blocks * 4;
}

void launch_mlp_reduce_adam(hipStream_t s, const float* ws, int nwaves, float* grad, float* loss, float* master,
                            float* m1, float* m2, u16* P, float lr, float beta1, float beta2, float eps, int step) {
    const float bc1 = 1.f - powf(beta1, (float)step), bc2 = 1.f - powf(beta2, (float)step);
    hipLaunchKernelGGL(k_mlp_reduce_adam, dim3((P_N + 1 + 255) / 256), dim3(256), 0, s, ws, nwaves, grad, loss,
                       master, m1, m2, P, lr, beta1, beta2, eps, bc1, bc2);
}

// workspace: network outputs (n x 4 floats), then two histograms of 256 bins
i64 calib_workspace_bytes(i64 n) { return 16 * n + 2 * 256 * 4; }

void launch_mlp_calibrate(hipStream_t s, const u16* X, const float* Y, i64 n, const u16* P, double max_false_accept,
                          double max_under_class, void* ws, u16* Q, double* shifts) {
    CalibGrid g;
    g.d[0] = 0.0;
    for (int k = 1; k < CalibGrid::K; ++k)  // geomspace(1e-3, 64, K - 1)
        g.d[k] = k == CalibGrid::K - 1 ? 64.0 : 1e-3 * pow(64.0 / 1e-3, (double)(k - 1) / (double)(CalibGrid::K - 2));
    float* out = static_cast<float*>(ws);
    u32* hist_a = reinterpret_cast<u32*>(static_cast<char*>(ws) + 16 * n);
    u32* hist_c = hist_a + 256;
    launch_fill_u32(s, hist_a, 512, 0u);
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (n > 0) launch_mlp_forward(s, X, n, nullptr, 0, P, out);
    if (n > 0) hipLaunchKernelGGL(k_calib_accept, dim3(blocks), dim3(256), 0, s, out, Y, n, g, hist_a);
    hipLaunchKernelGGL(k_calib_select, dim3(1), dim3(64), 0, s, hist_a, n, max_false_accept, g, 0, shifts);
    if (n > 0) hipLaunchKernelGGL(k_calib_class, dim3(blocks), dim3(256), 0, s, out, Y, n, g, shifts, hist_c);
    hipLaunchKernelGGL(k_calib_select, dim3(1), dim3(64), 0, s, hist_c, (i64)-1, max_under_class, g, 1, shifts);
    hipLaunchKernelGGL(k_calib_apply, dim3((P_N + 255) / 256), dim3(256), 0, s, P, shifts, Q);
}

void launch_mlp_batch_index(hipStream_t s, i64 n, i64 base, i64 nb, u64 a, u64 c, i32* idx) {
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_mlp_batch_index, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, n, base, nb, a, c, idx);
}

}  // namespace stc
