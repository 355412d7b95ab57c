// Training of the paper-size decoder (Sec. 4.2 "Decoder"; loss of Eq. (9)-(11))
// with one latent of 64 per fabric trained as a parameter.
//
//   paper_fwd_bwd_kernel   64 samples per block, wave w owning neurons
//                          16 w .. 16 w + 15 of every layer: one-blob
//                          features, the seven layers forward in FP32 (each
//                          layer's input vectors shared through LDS, its
//                          outputs also stored to the samples' planes), the
//                          loss terms and dL/dy, then the layers backward,
//                          storing every layer's gradient at its
//                          pre-activation
//   paper_wgrad_kernel     split-K weight gradients: per (job, chunk of
//                          256 samples) block, dL/dW and dL/db of one layer
//                          as sums of outer products over the chunk, staged
//                          through LDS 32 samples at a time, 4 x 4 entries
//                          per thread; one job sums F1's input gradient per
//                          fabric instead
//   paper_wgrad_reduce_kernel  fixed-order sum over the chunks
//   paper_latent_grads_kernel  F1's latent columns and the latents'
//                          gradients from the per-fabric sums
// Every reduction has a fixed order: results do not depend on scheduling.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "enc_dense.hpp"
#include "kernels.hpp"
#include "model.hpp"
#include "paper_net.hpp"
#include "paper_tile.hpp"
#include "paper_train.hpp"
#include "shade.hpp"
#include "train.hpp"

namespace fab {

namespace {

// Per-sample planes, each [cap] floats.
constexpr int kPlFeat = 0;              // 24 one-blob channels
constexpr int kPlAng = kPlFeat + 24;    // wi.xyz, wo.xy
constexpr int kPlT = kPlAng + 5;        // F1 activation (64)
constexpr int kPlSP = kPlT + 64;        // F2: the spatial feature
constexpr int kPlX = kPlSP + 64;        // A1: the residual block's input
constexpr int kPlH = kPlX + 64;         // A2
constexpr int kPlRR = kPlH + 64;        // A3 (skip added before its activation)
constexpr int kPlG = kPlRR + 64;        // A4
constexpr int kPlDY = kPlG + 64;        // dL/dy (4)
constexpr int kPlDT = kPlDY + 4;        // dL/d(pre-activation) of F1, F2, A1 .. A4
constexpr int kPlDSP = kPlDT + 64;
constexpr int kPlDX = kPlDSP + 64;
constexpr int kPlDH = kPlDX + 64;
constexpr int kPlDRR = kPlDH + 64;
constexpr int kPlDG = kPlDRR + 64;
constexpr int kPlanes = kPlDG + 64;
static_assert(kPlanes == 801, "plane count");

// BF16 training keeps the planes as BF16 values blocked by 64 samples: the
// 801 planes of samples 64 b .. 64 b + 63 form one contiguous region, each
// plane's 64 samples in order, so the weight gradients read eight
// consecutive samples of a plane with one 16-byte load and a chunk's reads
// stay within its regions.
constexpr int kQBlock = 64;
__host__ __device__ inline int64_t q_elem(int plane, int64_t s)
{
    // s >= 0: the shift and the mask are the quotient and the remainder.
    return (s >> 6) * ((int64_t)kPlanes * kQBlock) + plane * kQBlock + (s & (kQBlock - 1));
}

// Transposed weights of every layer for the forward pass, WT[i][o] =
// W[o][i] (the 16 outputs of a wave are then 16 consecutive floats).
enum { kTF1 = 0, kTF2, kTA1, kTA2, kTA3, kTA4, kTA5, kTLayers };
__host__ __device__ constexpr int t_in(int l) { return l == kTF1 ? kPX1 : l == kTA1 ? kPXA1 : 64; }
__host__ __device__ constexpr int t_out(int l) { return l == kTA5 ? 4 : 64; }
__host__ __device__ constexpr int t_first(int l)
{
    return l == 0 ? 0 : t_first(l - 1) + t_in(l - 1) * t_out(l - 1);
}
constexpr int kTFloats = t_first(kTLayers);          // 26,688
__host__ __device__ constexpr int w_off(int l)
{
    return l == kTF1 ? kPOffWF1 : l == kTF2 ? kPOffWF2 : l == kTA1 ? kPOffWA1 : l == kTA2 ? kPOffWA2
           : l == kTA3 ? kPOffWA3 : l == kTA4 ? kPOffWA4 : kPOffWA5;
}

__global__ void transpose_kernel(const float *__restrict__ P, float *__restrict__ wt)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= kTFloats)
        return;
    int l = 0;
    while (l + 1 < kTLayers && idx >= t_first(l + 1))
        l++;
    const int k = idx - t_first(l), i = k / t_out(l), o = k % t_out(l);
    wt[idx] = P[w_off(l) + o * t_in(l) + i];
}


// The forward and backward pass of 64 samples per block: lane l of every
// wave owns sample 64 b + l, and wave w owns neurons 16 w .. 16 w + 15 of each
// 64-wide layer (weights read as wave-uniform scalars).  A layer's input
// vector of each sample is shared through LDS; every value a wave needs from
// its own earlier work (activations for the slopes, the residual input) is
// its own.  Activations and gradients also go to the per-sample planes.
constexpr int kFbSamples = 64;
constexpr int kFbStride = kPX1 + 1;                  // LDS row of one sample (odd: no conflicts)
constexpr int kFbStrideB = 64 + 1;                   // the second buffer holds at most 64 per sample

// acc[k] = b[o] + sum_i WT[i][o] x[i] for o = o0 + k (WT: [NIN][NOUT]).
template <int NIN, int NOUT>
__device__ inline void fwd16(const float *__restrict__ WT, const float *__restrict__ b,
                             const float *xrow, int o0, float (&acc)[16])
{
#pragma unroll
    for (int k = 0; k < 16; k++)
        acc[k] = b[o0 + k];
#pragma unroll 8
    for (int i = 0; i < NIN; i++) {
        const float xi = xrow[i];
#pragma unroll
        for (int k = 0; k < 16; k++)
            acc[k] = fmaf(WT[i * NOUT + o0 + k], xi, acc[k]);
    }
}

// acc[k] = sum_o W[o][i] g[o] for i = i0 + k (W row-major [NG][ROW]).
template <int NG, int ROW>
__device__ inline void bwd16(const float *__restrict__ W, const float *grow, int i0,
                             float (&acc)[16])
{
#pragma unroll
    for (int k = 0; k < 16; k++)
        acc[k] = 0.0f;
#pragma unroll 8
    for (int o = 0; o < NG; o++) {
        const float go = grow[o];
#pragma unroll
        for (int k = 0; k < 16; k++)
            acc[k] = fmaf(W[o * ROW + i0 + k], go, acc[k]);
    }
}

// Four blocks per CU (at most 128 VGPRs, under 40 KB of LDS per block): a
// 2^16-sample batch is then one round of 1,024 blocks.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void paper_fwd_bwd_kernel(
    fabric_gbuffer g, const DevFabric *__restrict__ fabrics, int n_fabrics,
    const float *__restrict__ P, const float *__restrict__ lat, const float *__restrict__ wt,
    const float *__restrict__ targets, float *__restrict__ pl, int64_t cap, int raw, int fused,
    float *__restrict__ loss_part)
{
    __shared__ float bufA[kFbSamples * kFbStride];
    __shared__ float bufB[kFbSamples * kFbStrideB];
    __shared__ float red[kFbSamples];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int o0 = 16 * w;
    const int64_t n = g.n;
    const int64_t s = (int64_t)blockIdx.x * kFbSamples + lane;
    const bool live = s < n;
    int fid = 0;
    float u = 0.0f, v = 0.0f, r = 1.0f;
    float3 wi = make_float3(0.0f, 0.0f, 1.0f), wo = make_float3(0.0f, 0.0f, 1.0f);
    if (live) {
        fid = g.fabric_id[s];
        u = g.u[s]; v = g.v[s]; r = g.radius[s];
        wi = make_float3(g.wi_x[s], g.wi_y[s], g.wi_z[s]);
        wo = make_float3(g.wo_x[s], g.wo_y[s], g.wo_z[s]);
    }
    // A faulted sample contributes nothing: it runs on harmless inputs and
    // stores zeros to every plane.
    const bool fault = !live || pixel_fault(fid, n_fabrics, u, v, r, wi, wo);
    if (fault) {
        fid = 0; u = 0.0f; v = 0.0f; r = 1.0f;
        wi = make_float3(0.0f, 0.0f, 1.0f);
        wo = make_float3(0.0f, 0.0f, 1.0f);
    }
    auto store = [&](int plane, float val) {
        if (live)
            pl[(int64_t)plane * cap + s] = fault ? 0.0f : val;
    };
    float *rowA = bufA + lane * kFbStride, *rowB = bufB + lane * kFbStrideB;
    const float ang[5] = {wi.x, wi.y, wi.z, wo.x, wo.y};

    // ---- F1 input [z, one-blob] (each wave fills a quarter of the row) ----
#pragma unroll
    for (int k = 0; k < 16; k++)
        rowA[o0 + k] = lat[fid * kPLat + o0 + k];
    if (w == 0) {
        float f[24];
        blob24(fabrics[fid], u, v, r, raw != 0, f);
#pragma unroll
        for (int k = 0; k < 24; k++) {
            rowA[kPLat + k] = f[k];
            store(kPlFeat + k, f[k]);
        }
#pragma unroll
        for (int k = 0; k < 5; k++)
            store(kPlAng + k, ang[k]);
    }
    __syncthreads();
    float acc[16], xres[16];
    // A forward layer: outputs of this wave's neurons, activated (+ skip),
    // to the other buffer and the plane.
    // Without the spatial fusion stage the angular inputs enter F1 through
    // A1's angular columns (add_ang).
    // The signs of this wave's activations (bit k: neuron o0 + k > 0), kept
    // for the backward pass's slopes.
    auto layer = [&](auto nin_tag, int tl, const float *bias, const float *in, float *out, int plane,
                     bool skip, bool add_ang, uint32_t &pos) {
        constexpr int NIN = decltype(nin_tag)::value;
        fwd16<NIN, 64>(wt + t_first(tl), bias, in, o0, acc);
        if (add_ang) {
#pragma unroll
            for (int k = 0; k < 16; k++)
#pragma unroll
                for (int a = 0; a < 5; a++)
                    acc[k] = fmaf(P[kPOffWA1 + (o0 + k) * kPXA1 + 64 + a], ang[a], acc[k]);
        }
        pos = 0u;
#pragma unroll
        for (int k = 0; k < 16; k++) {
            const float a = lrelu(skip ? acc[k] + xres[k] : acc[k]);
            out[o0 + k] = a;
            store(plane + o0 + k, a);
            acc[k] = a;
            pos |= (a > 0.0f ? 1u : 0u) << k;
        }
        __syncthreads();
    };
    using I88 = std::integral_constant<int, kPX1>;
    using I69 = std::integral_constant<int, kPXA1>;
    using I64 = std::integral_constant<int, 64>;
    uint32_t pT, pSP, pX, pH, pRR, pG;
    layer(I88{}, kTF1, P + kPOffBF1, rowA, rowB, kPlT, false, fused == 0, pT);
    layer(I64{}, kTF2, P + kPOffBF2, rowB, rowA, kPlSP, false, false, pSP);
    if (w == 0) {
#pragma unroll
        for (int k = 0; k < 5; k++)
            rowA[64 + k] = fused ? ang[k] : 0.0f;
    }
    __syncthreads();
    layer(I69{}, kTA1, P + kPOffBA1, rowA, rowB, kPlX, false, false, pX);
#pragma unroll
    for (int k = 0; k < 16; k++)
        xres[k] = acc[k];                               // the residual block's input
    layer(I64{}, kTA2, P + kPOffBA2, rowB, rowA, kPlH, false, false, pH);
    layer(I64{}, kTA3, P + kPOffBA3, rowA, rowB, kPlRR, true, false, pRR);
    layer(I64{}, kTA4, P + kPOffBA4, rowB, rowA, kPlG, false, false, pG);
    // ---- A5: wave w computes output w; the four meet in LDS ----
    {
        float y = P[kPOffBA5 + w];
        const float *WT5 = wt + t_first(kTA5);
#pragma unroll 8
        for (int i = 0; i < 64; i++)
            y = fmaf(WT5[i * 4 + w], rowA[i], y);
        rowB[w] = y;
    }
    __syncthreads();
    // ---- loss terms of Eq. (9)-(11) and dL/dy (every wave, for its own use) ----
    float dy[4];
    float loss = 0.0f;
    {
        const float inv_n = 1.0f / (float)n;
        // g(x) = ln(k x + 1): k = 100 for reflection, 1000 for transmission.
        const float k = wi.z < 0.0f ? 10.0f * kSpec : kSpec;
#pragma unroll
        for (int c = 0; c < 4; c++) {
            const float t = fault ? 0.0f : targets[c * n + s];
            const float target = c < 2 ? t : log1pf(k * t);
            const float lam = c < 2 ? 0.1f : 0.4f;        // lambda_C, lambda_S
            const float d = rowB[c] - target;
            loss = fault ? loss : fmaf(lam * d, d, loss);
            dy[c] = fault ? 0.0f : 2.0f * lam * d * inv_n;
        }
        if (w == 0) {
#pragma unroll
            for (int c = 0; c < 4; c++)
                store(kPlDY + c, dy[c]);
        }
    }
    __syncthreads();                                    // rowB's outputs read by all
    // ---- backward: this wave's 16 input gradients of each layer ----
    auto back = [&](auto ng_tag, auto row_tag, int woff, const float *gin, float *gout,
                    uint32_t pos, int out_plane, const float *extra) {
        constexpr int NG = decltype(ng_tag)::value;
        constexpr int ROW = decltype(row_tag)::value;
        bwd16<NG, ROW>(P + woff, gin, o0, acc);
#pragma unroll
        for (int k = 0; k < 16; k++) {
            const float t = extra ? acc[k] + extra[k] : acc[k];
            const float d = (pos >> k) & 1u ? t : kLeak * t;
            acc[k] = fault ? 0.0f : d;
            gout[o0 + k] = acc[k];
            store(out_plane + o0 + k, acc[k]);
        }
        __syncthreads();
    };
    using I4 = std::integral_constant<int, 4>;
    back(I4{}, I64{}, kPOffWA5, dy, rowA, pG, kPlDG, nullptr);
    back(I64{}, I64{}, kPOffWA4, rowA, rowB, pRR, kPlDRR, nullptr);
    float drr[16];
#pragma unroll
    for (int k = 0; k < 16; k++)
        drr[k] = acc[k];                                // the skip's gradient to A1's output
    back(I64{}, I64{}, kPOffWA3, rowB, rowA, pH, kPlDH, nullptr);
    back(I64{}, I64{}, kPOffWA2, rowA, rowB, pX, kPlDX, drr);
    back(I64{}, I69{}, kPOffWA1, rowB, rowA, pSP, kPlDSP, nullptr);
    back(I64{}, I64{}, kPOffWF2, rowA, rowB, pT, kPlDT, nullptr);

    // Fixed-order sum of the block's loss terms (wave 0 holds them).
    if (w == 0)
        red[lane] = loss;
    __syncthreads();
    if (threadIdx.x == 0) {
        KahanSum t;
        for (int k = 0; k < kFbSamples; k++)
            t.add(red[k]);
        loss_part[blockIdx.x] = t.value();
    }
}

__global__ __launch_bounds__(256) void paper_loss_reduce_kernel(const float *__restrict__ part,
                                                                int64_t nparts, float inv_n,
                                                                float *__restrict__ loss)
{
    __shared__ float red[256];
    KahanSum acc;
    for (int64_t k = threadIdx.x; k < nparts; k += blockDim.x)
        acc.add(part[k]);
    red[threadIdx.x] = acc.value();
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        loss[0] = red[0] * inv_n;
}

// ---- BF16 operands on MFMA (cfg.prec == FABRIC_BF16) ----------------------
//
// The forward runs the shading kernel's tile (paper_tile.hpp) on the BF16
// shading image that the masters were last packed into, 32 samples per wave,
// with its scaled activations; the backward chains the transposed weights
// the same way: the gradient at a layer's pre-activation, held in the
// accumulator layout, is the B operand of the next transposed layer without
// data movement.  The quantities of the FP32 path's planes (s times the
// scaled activations: the FP32 network's activations to FP32 rounding; the
// gradients) go to BF16 planes blocked by 64 samples (q_elem), whose weight
// gradients paper_wgrad_bf16_kernel sums.
//
// Transposed-weight fragments, in the order the backward uses them: A5^T
// (2 M-blocks, one K step: the four outputs in slots 0..3 of lane group 0),
// then A4^T, A3^T, A2^T, A1^T (its 64 spatial columns) and F2^T (2 M-blocks
// x 4 K steps of chained neurons each).
enum { kBA5 = 0, kBA4, kBA3, kBA2, kBA1, kBF2, kBLayers };
__host__ __device__ constexpr int bwd_first(int l) { return l == 0 ? 0 : 2 + (l - 1) * 8; }
constexpr int kBFrags = bwd_first(kBLayers);       // 42
static_assert(kBFrags == 42, "backward fragment count");

__global__ void pack_paper_bwd_kernel(const float *__restrict__ P, bf16x8 *__restrict__ frags)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= kBFrags * 64)
        return;
    const int fr = idx / 64, lane = idx % 64, row = lane & 31, grp = lane >> 5;
    int layer = 0, mb = fr, ks = 0;
    if (fr >= 2) {
        layer = 1 + (fr - 2) / 8;
        mb = ((fr - 2) % 8) / 4;
        ks = (fr - 2) % 4;
    }
    const int m = 32 * mb + row;                    // input neuron of the forward layer
    const int woff = layer == kBA4 ? kPOffWA4 : layer == kBA3 ? kPOffWA3 : layer == kBA2 ? kPOffWA2
                     : layer == kBA1 ? kPOffWA1 : kPOffWF2;
    const int row_len = layer == kBA1 ? kPXA1 : 64;
    f32x8 w;
    for (int j = 0; j < 8; j++) {
        const int c = ks * 8 + j;
        if (layer == kBA5)
            w[j] = grp == 0 && c < 4 ? P[kPOffWA5 + c * 64 + m] : 0.0f;
        else
            w[j] = P[woff + chain32_neuron(grp, c) * row_len + m];
    }
    frags[idx] = Mfma<FABRIC_BF16>::from8(w);
}

// Forward, loss and backward of 32 samples per wave, four waves per block
// (128 samples per block: one loss part each).
template <bool RAW, bool FUSED>
__global__ __launch_bounds__(256, 2) void paper_fwd_bwd_bf16_kernel(
    fabric_gbuffer g, const DevFabric *__restrict__ fabrics, int n_fabrics,
    const float *__restrict__ cfold, const bf16x8 *__restrict__ ffr, const f32x4 *__restrict__ bias5,
    const bf16x8 *__restrict__ bfr, const float *__restrict__ targets, float *__restrict__ pl,
    float *__restrict__ loss_part)
{
    using PT = PaperTile<FABRIC_BF16>;
    using M = typename PT::M;
    using Frag = bf16x8;
    // LDS: per fabric c_f [64], then the staged constants.
    extern __shared__ f32x4 smem4[];
    float *s_cf = (float *)smem4;
    float *s_fc = s_cf + n_fabrics * 64;
    __shared__ float red[4];
    for (int k = threadIdx.x; k < n_fabrics * 64; k += blockDim.x)
        s_cf[k] = cfold[k];
    stage_fabric_consts(fabrics, n_fabrics, s_fc);
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int grp = lane >> 5;
    const int col = lane & 31;
    const int w = threadIdx.x >> 6;
    const int64_t n = g.n;
    const int64_t s = ((int64_t)blockIdx.x * 4 + w) * 32 + col;   // this lane's sample
    const bool live = s < n;
    const uint32_t dmask = half_dir_mask(grp);
    HalfPix cur = load_half(g, half_planes(g, grp), (int)(live ? s : n - 1));
    // A faulted sample contributes nothing: it runs on harmless inputs and
    // stores zeros to every plane.
    const bool fault = !live || pair_any(half_fault(cur, n_fabrics, dmask));
    if (fault) {
        cur.fid = 0;
        cur.uv = 0.0f;
        cur.r = 1.0f;
        cur.x0 = 0.0f;
        cur.x1 = 0.0f;
        cur.xz = 1.0f;
    }
    // The BF16 planes (blocked by 64 samples) in the buffer of the FP32 ones.
    __bf16 *qp = (__bf16 *)pl;
    auto store = [&](int plane, float val) {
        if (live)
            qp[q_elem(plane, s)] = (__bf16)(fault ? 0.0f : val);
    };
    // Accumulator register r of M-block mb holds neuron 32 mb + 8 (r/4) + 4 g + r%4.
    auto store_acc = [&](int plane, const f32x16 (&v)[2]) {
#pragma unroll
        for (int mb = 0; mb < 2; mb++)
#pragma unroll
            for (int r = 0; r < 16; r++)
                store(plane + 32 * mb + 8 * (r >> 2) + 4 * grp + (r & 3), v[mb][r]);
    };
    // A layer's output v in place: the scaled activation that the image
    // expects (as the shading tile computes it), and plane_s times it - the
    // FP32 network's activation - to `plane`; bit mb*16 + r of the returned
    // mask: positive.
    auto activate = [&](int plane, f32x16 (&v)[2], float plane_s) {
        uint32_t pos = 0u;
#pragma unroll
        for (int mb = 0; mb < 2; mb++)
#pragma unroll
            for (int r = 0; r < 16; r++) {
                pos |= (v[mb][r] > 0.0f ? 1u : 0u) << (16 * mb + r);
                v[mb][r] = lrelu_scaled(v[mb][r]);
            }
#pragma unroll
        for (int mb = 0; mb < 2; mb++)
#pragma unroll
            for (int r = 0; r < 16; r++)
                store(plane + 32 * mb + 8 * (r >> 2) + 4 * grp + (r & 3), plane_s * v[mb][r]);
        return pos;
    };
    // The leaky ReLU's slope applied to a gradient at the activation.
    auto slope = [&](f32x16 (&d)[2], uint32_t pos) {
#pragma unroll
        for (int mb = 0; mb < 2; mb++)
#pragma unroll
            for (int r = 0; r < 16; r++)
                d[mb][r] = (pos >> (16 * mb + r)) & 1u ? d[mb][r] : kLeak * d[mb][r];
    };
    f32x8 one8 = {grp == 0 ? 1.0f : 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    const Frag bias_b = M::from8(one8);

    // ---- forward ----
    const int entry = fab_entry(cur.fid, n_fabrics, grp ? 1.0f : cur.xz);
    const float *fc = s_fc + entry * kFabConsts;
    f32x16 a[1][2];
    {
        float s1[FUSED ? kPSlots1 : kPSlots1 + 4];
        const float per = grp ? fc[1] : fc[0], iper = grp ? fc[3] : fc[2];
        paper_slots<FABRIC_BF16, RAW>(wrap_period(cur.uv, per, iper), iper, cur.r, grp, s1);
        if (!FUSED) {
            s1[kPSlots1] = cur.x0;
            s1[kPSlots1 + 1] = cur.x1;
            s1[kPSlots1 + 2] = grp ? 0.0f : cur.xz;
        }
#pragma unroll
        for (int c = 0; c < kPSlots1; c++)
            store(kPlFeat + p_blob_channel(grp, c), s1[c]);
        if (grp == 0) {
            store(kPlAng + 0, cur.x0);
            store(kPlAng + 1, cur.x1);
            store(kPlAng + 2, cur.xz);
        } else {
            store(kPlAng + 3, cur.x0);
            store(kPlAng + 4, cur.x1);
        }
        Frag B1[1][2];
        B1[0][0] = PT::frag_of(s1, 0, false);
        B1[0][1] = PT::frag_of(s1, 1, false);
#pragma unroll
        for (int mb = 0; mb < 2; mb++)
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const f32x4 c4 = *(const f32x4 *)(s_cf + cur.fid * 64 + 32 * mb + 8 * q + 4 * grp);
#pragma unroll
                for (int i = 0; i < 4; i++)
                    a[0][mb][4 * q + i] = c4[i];
            }
        PT::template dense_lds<1, 2, 2>(ffr, p_first(kF1), B1, a, lane);
    }
    // The chained B operand of an activated 64-neuron output and its bias step.
    auto chain_in = [&](Frag (&B)[1][5]) {
        Frag B4[4];
        PT::chain_b(a[0], B4, false);
#pragma unroll
        for (int ks = 0; ks < 4; ks++)
            B[0][ks] = B4[ks];
        B[0][4] = bias_b;
    };
    auto chain_layer = [&](int layer) {
        Frag B[1][5];
        chain_in(B);
        a[0][0] = a[0][1] = f32x16{};
        PT::template dense_lds<1, 2, 5>(ffr, p_first(layer), B, a, lane);
    };
    const uint32_t pT = activate(kPlT, a[0], kActS);
    chain_layer(kF2);
    const uint32_t pSP = activate(kPlSP, a[0], kActS);
    {
        // A1: [spatial feature, wi.xyz | wo.xy, 1]
        Frag B[1][5];
        float v[kL3Slots32];
#pragma unroll
        for (int c = 0; c < kChain32; c++)
            v[c] = a[0][c >> 4][c & 15];
        v[32] = cur.x0;
        v[33] = cur.x1;
        v[34] = grp ? 1.0f : cur.xz;
#pragma unroll
        for (int ks = 0; ks < 5; ks++)
            B[0][ks] = PT::frag_of(v, ks, false);
        a[0][0] = a[0][1] = f32x16{};
        PT::template dense_lds<1, 2, 5>(ffr, p_first(kA1), B, a, lane);
    }
    const uint32_t pX = activate(kPlX, a[0], kActS);
    f32x16 x[1][2] = {{a[0][0], a[0][1]}};              // the residual block's input
    chain_layer(kA2);
    const uint32_t pH = activate(kPlH, a[0], kActS);
    {
        // A3 from C operand x: the skip enters before the activation.
        Frag B[1][5];
        chain_in(B);
        PT::template dense_lds<1, 2, 5>(ffr, p_first(kA3), B, x, lane);
        a[0][0] = x[0][0];
        a[0][1] = x[0][1];
    }
    const uint32_t pRR = activate(kPlRR, a[0], kActS * kActS);  // A3's output at scale 1/s
    chain_layer(kA4);
    const uint32_t pG = activate(kPlG, a[0], kActS);
    {
        // A5: four outputs in rows 0..3 (lane group 0), bias added after.
        Frag B[1][4];
        PT::chain_b(a[0], B[0], false);
        a[0][0] = f32x16{};
        PT::template dense_lds<1, 1, 4>(ffr, p_first(kA5), B, a, lane);
    }

    // ---- loss terms of Eq. (9)-(11) and dL/dy (lane group 0 holds y) ----
    const f32x4 b5 = bias5[lane];
    float dy[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    float loss = 0.0f;
    if (grp == 0 && !fault) {
        const float inv_n = 1.0f / (float)n;
        // g(x) = ln(k x + 1): k = 100 for reflection, 1000 for transmission.
        const float k = cur.xz < 0.0f ? 10.0f * kSpec : kSpec;
#pragma unroll
        for (int c = 0; c < 4; c++) {
            const float t = targets[c * n + s];
            const float target = c < 2 ? t : log1pf(k * t);
            const float lam = c < 2 ? 0.1f : 0.4f;        // lambda_C, lambda_S
            const float d = a[0][0][c] + b5[c] - target;
            loss = fmaf(lam * d, d, loss);
            dy[c] = 2.0f * lam * d * inv_n;
        }
    }
    if (grp == 0) {
#pragma unroll
        for (int c = 0; c < 4; c++)
            store(kPlDY + c, dy[c]);
    }

    // ---- backward ----
    f32x16 d[2];
    {
        const f32x8 v = {dy[0], dy[1], dy[2], dy[3], 0.0f, 0.0f, 0.0f, 0.0f};
        const Frag B = M::from8(v);                      // zero in lane group 1
#pragma unroll
        for (int mb = 0; mb < 2; mb++)
            d[mb] = Mfma32<FABRIC_BF16>::mma(bfr[(bwd_first(kBA5) + mb) * 64 + lane], B, f32x16{});
    }
    // d <- (W^T d) of one chained layer, C operand c.
    auto back = [&](int layer, const f32x16 (&c)[2]) {
        Frag B[4];
        PT::chain_b(d, B, false);
#pragma unroll
        for (int mb = 0; mb < 2; mb++) {
            f32x16 acc = c[mb];
#pragma unroll
            for (int ks = 0; ks < 4; ks++)
                acc = Mfma32<FABRIC_BF16>::mma(bfr[(bwd_first(layer) + 4 * mb + ks) * 64 + lane],
                                               B[ks], acc);
            d[mb] = acc;
        }
    };
    const f32x16 zero2[2] = {f32x16{}, f32x16{}};
    slope(d, pG);
    store_acc(kPlDG, d);
    back(kBA4, zero2);
    slope(d, pRR);
    store_acc(kPlDRR, d);
    const f32x16 drr[2] = {d[0], d[1]};                  // the skip's gradient to A1's output
    back(kBA3, zero2);
    slope(d, pH);
    store_acc(kPlDH, d);
    back(kBA2, drr);
    slope(d, pX);
    store_acc(kPlDX, d);
    back(kBA1, zero2);
    slope(d, pSP);
    store_acc(kPlDSP, d);
    back(kBF2, zero2);
    slope(d, pT);
    store_acc(kPlDT, d);

    // ---- the block's loss: lane group 0 of each wave, then the waves in order ----
#pragma unroll
    for (int off = 16; off > 0; off >>= 1)
        loss += __shfl_xor(loss, off, 64);
    if (lane == 0)
        red[w] = loss;
    __syncthreads();
    if (threadIdx.x == 0) {
        KahanSum t;
        for (int k = 0; k < 4; k++)
            t.add(red[k]);
        loss_part[blockIdx.x] = t.value();
    }
}

// ---- split-K weight gradients ----------------------------------------------

// One job: out[i][j] = sum_s delta_i(s) in_j(s) over i < n_out and the
// inputs [planes inA .. inA + nA, inB .. inB + nB, then 1 for the bias when
// b_off >= 0]; or, for the one-hot job, in_j(s) = [fabric id of s == j].
struct PWJob {
    int delta, n_out, inA, nA, inB, nB;
    int w_off, row, col, b_off;     // destination in the parameter gradient
    int onehot;                     // 1: per-fabric sums into dsum[j][i]
};
constexpr int kPWMaxJobs = 9;
struct PWJobs {
    PWJob j[kPWMaxJobs];
    int64_t poff[kPWMaxJobs];       // job offsets in the partial buffer
    int n_jobs;
};

constexpr int kPwChunk = 512;       // samples per block
constexpr int kPwMaxIn = 70;        // columns (inputs + bias) of any job
constexpr int kPwColBlocks = 5;     // 16-column blocks of the widest job
static_assert(kPwMaxIn <= 16 * kPwColBlocks, "column blocks");
constexpr int kPwThreads = 256;     // one 16-row block of outputs per wave

__host__ __device__ inline int pw_cols(const PWJob &jb)
{
    return jb.nA + jb.nB + (jb.b_off >= 0 ? 1 : 0);
}

// Weight gradients on FP32 MFMA 16x16x4, samples being the K dimension: a
// block takes one job and one chunk of kPwChunk samples, wave w the output
// rows 16 w .. 16 w + 15 for every 16-column block of the job.  Lane
// (q = l/16, c = l%16) reads samples s + 8 q .. s + 8 q + 7 of its row's
// delta plane and of its columns' input planes as two float4s (the planes
// are sample-contiguous, their stride a multiple of 64), and MFMA t of a
// group of 32 samples takes sample s + 8 q + t in k slot q.  A job's column
// blocks but the last hold input planes only; the last mixes planes, the
// bias column (1) and padding (0).  Samples past the batch (stale plane
// values) enter as zeros in both operands.
struct PwLane {
    const float *a;                 // the lane's delta row (nullptr: a padding row)
    const float *b[kPwColBlocks];   // input planes of the lane's columns
    bool b_plane;                   // the last block's column is a plane
    float b_const;                  // else its value (1 for the bias, 0 for padding)
    const uint16_t *fid;            // one-hot job: the fabric ids
};

template <int CB, bool ONEHOT, bool TAIL>
__device__ inline void pw_group(const PwLane &L, int c, int64_t base, int64_t s1, f32x4 (&acc)[CB])
{
    auto in = [&](int t) { return !TAIL || base + t < s1; };
    float a[8];
    if (L.a) {
        const f32x4 lo = *(const f32x4 *)(L.a + base), hi = *(const f32x4 *)(L.a + base + 4);
#pragma unroll
        for (int t = 0; t < 4; t++) {
            a[t] = in(t) ? lo[t] : 0.0f;
            a[4 + t] = in(4 + t) ? hi[t] : 0.0f;
        }
    } else {
#pragma unroll
        for (int t = 0; t < 8; t++)
            a[t] = 0.0f;
    }
    float b[CB][8];
    if (ONEHOT) {
        int id[8];
#pragma unroll
        for (int t = 0; t < 8; t++)
            id[t] = in(t) ? (int)L.fid[base + t] : -1;
#pragma unroll
        for (int cb = 0; cb < CB; cb++)
#pragma unroll
            for (int t = 0; t < 8; t++)
                b[cb][t] = id[t] == 16 * cb + c ? 1.0f : 0.0f;
    } else {
#pragma unroll
        for (int cb = 0; cb < CB; cb++) {
            const f32x4 lo = *(const f32x4 *)(L.b[cb] + base);
            const f32x4 hi = *(const f32x4 *)(L.b[cb] + base + 4);
            const bool plane = cb < CB - 1 || L.b_plane;
#pragma unroll
            for (int t = 0; t < 4; t++) {
                b[cb][t] = plane ? (in(t) ? lo[t] : 0.0f) : L.b_const;
                b[cb][4 + t] = plane ? (in(4 + t) ? hi[t] : 0.0f) : L.b_const;
            }
        }
    }
#pragma unroll
    for (int t = 0; t < 8; t++)
#pragma unroll
        for (int cb = 0; cb < CB; cb++)
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t], b[cb][t], acc[cb], 0, 0, 0);
}

template <int CB, bool ONEHOT>
__device__ inline void pw_chunk(const PwLane &L, const PWJob &jb, int cols, int w, int q, int c,
                                int64_t s0, int64_t s1, float *__restrict__ dst)
{
    f32x4 acc[CB];
#pragma unroll
    for (int cb = 0; cb < CB; cb++)
        acc[cb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    int64_t sb = s0;
    for (; sb + 32 <= s1; sb += 32)
        pw_group<CB, ONEHOT, false>(L, c, sb + 8 * q, s1, acc);
    if (sb < s1)
        pw_group<CB, ONEHOT, true>(L, c, sb + 8 * q, s1, acc);
    // Register i of a tile holds row 4 q + i, column c.
#pragma unroll
    for (int cb = 0; cb < CB; cb++) {
        const int j = 16 * cb + c;
        if (j >= cols)
            continue;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int r = 16 * w + 4 * q + i;
            if (r < jb.n_out)
                dst[r * cols + j] = acc[cb][i];
        }
    }
}

__global__ __launch_bounds__(kPwThreads) void paper_wgrad_kernel(PWJobs jobs,
                                                                 const float *__restrict__ pl,
                                                                 int64_t cap,
                                                                 const uint16_t *__restrict__ fid,
                                                                 int64_t n,
                                                                 float *__restrict__ partial)
{
    const PWJob jb = jobs.j[blockIdx.y];
    const int cols = pw_cols(jb);
    const int lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
    const int w = threadIdx.x >> 6;
    if (16 * w >= jb.n_out)
        return;
    const int cb_n = (cols + 15) >> 4;
    const int row = 16 * w + c;
    PwLane L;
    L.a = row < jb.n_out ? pl + (int64_t)(jb.delta + row) * cap : nullptr;
    L.fid = fid;
    L.b_plane = false;
    L.b_const = 0.0f;
#pragma unroll
    for (int cb = 0; cb < kPwColBlocks; cb++) {
        const int j = 16 * cb + c;
        // A column that is no plane reads the first input plane (in bounds)
        // and takes its constant instead.
        int plane = jb.inA;
        if (j < jb.nA)
            plane = jb.inA + j;
        else if (j < jb.nA + jb.nB)
            plane = jb.inB + j - jb.nA;
        L.b[cb] = pl + (int64_t)plane * cap;
        if (cb == cb_n - 1) {
            L.b_plane = j < jb.nA + jb.nB;
            L.b_const = j < cols ? 1.0f : 0.0f;     // the bias column, or padding
        }
    }
    const int64_t s0 = (int64_t)blockIdx.x * kPwChunk;
    const int64_t s1 = s0 + kPwChunk < n ? s0 + kPwChunk : n;
    float *dst = partial + jobs.poff[blockIdx.y] + (int64_t)blockIdx.x * jb.n_out * cols;
    if (jb.onehot) {
        switch (cb_n) {
        case 1: pw_chunk<1, true>(L, jb, cols, w, q, c, s0, s1, dst); break;
        case 2: pw_chunk<2, true>(L, jb, cols, w, q, c, s0, s1, dst); break;
        case 3: pw_chunk<3, true>(L, jb, cols, w, q, c, s0, s1, dst); break;
        default: pw_chunk<4, true>(L, jb, cols, w, q, c, s0, s1, dst); break;
        }
        return;
    }
    switch (cb_n) {
    case 1: pw_chunk<1, false>(L, jb, cols, w, q, c, s0, s1, dst); break;
    case 2: pw_chunk<2, false>(L, jb, cols, w, q, c, s0, s1, dst); break;
    case 3: pw_chunk<3, false>(L, jb, cols, w, q, c, s0, s1, dst); break;
    case 4: pw_chunk<4, false>(L, jb, cols, w, q, c, s0, s1, dst); break;
    default: pw_chunk<5, false>(L, jb, cols, w, q, c, s0, s1, dst); break;
    }
}

// The same jobs from the BF16 planes of BF16 training, on BF16 MFMA
// 16x16x32: lane (q = l/16, c = l%16) holds samples s + 8 q .. s + 8 q + 7 of
// its delta row and of its columns' planes (one 16-byte load each, within
// one 64-sample region), which fill k slots 8 q .. 8 q + 7 of both operands
// alike; one MFMA per 16-column block and group of 32 samples.
struct PqLane {
    const __bf16 *qp;               // the planes
    int a;                          // the lane's delta plane (-1: a padding row)
    int b[kPwColBlocks];            // input planes of the lane's columns
    bool b_plane;                   // the last block's column is a plane
    __bf16 b_const;                 // else its value (1 for the bias, 0 for padding)
    const uint16_t *fid;            // one-hot job: the fabric ids
};

// The operands of one group of 32 samples.
template <int CB> struct PqOps {
    bf16x8 a;
    bf16x8 b[CB];
};

template <int CB, bool ONEHOT, bool TAIL>
__device__ inline void pq_load(const PqLane &L, int c, int64_t base, int64_t s1, PqOps<CB> &o)
{
    const __bf16 zero = (__bf16)0.0f, one = (__bf16)1.0f;
    auto in = [&](int t) { return !TAIL || base + t < s1; };
    const __bf16 *reg = L.qp + q_elem(0, base);
    if (L.a >= 0) {
        o.a = *(const bf16x8 *)(reg + L.a * kQBlock);
        if (TAIL) {
#pragma unroll
            for (int t = 0; t < 8; t++)
                o.a[t] = in(t) ? o.a[t] : zero;
        }
    } else {
#pragma unroll
        for (int t = 0; t < 8; t++)
            o.a[t] = zero;
    }
    if (ONEHOT) {
        int id[8];
#pragma unroll
        for (int t = 0; t < 8; t++)
            id[t] = in(t) ? (int)L.fid[base + t] : -1;
#pragma unroll
        for (int cb = 0; cb < CB; cb++)
#pragma unroll
            for (int t = 0; t < 8; t++)
                o.b[cb][t] = id[t] == 16 * cb + c ? one : zero;
    } else {
#pragma unroll
        for (int cb = 0; cb < CB; cb++) {
            const bf16x8 v = *(const bf16x8 *)(reg + L.b[cb] * kQBlock);
            const bool plane = cb < CB - 1 || L.b_plane;
#pragma unroll
            for (int t = 0; t < 8; t++)
                o.b[cb][t] = plane ? (in(t) ? v[t] : zero) : L.b_const;
        }
    }
}

template <int CB>
__device__ inline void pq_mma(const PqOps<CB> &o, f32x4 (&acc)[CB])
{
#pragma unroll
    for (int cb = 0; cb < CB; cb++)
        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(o.a, o.b[cb], acc[cb], 0, 0, 0);
}

template <int CB, bool ONEHOT>
__device__ inline void pq_chunk(const PqLane &L, const PWJob &jb, int cols, int w, int q, int c,
                                int64_t s0, int64_t s1, float *__restrict__ dst)
{
    f32x4 acc[CB];
#pragma unroll
    for (int cb = 0; cb < CB; cb++)
        acc[cb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    int64_t sb = s0;
    for (; sb + 32 <= s1; sb += 32) {
        PqOps<CB> o;
        pq_load<CB, ONEHOT, false>(L, c, sb + 8 * q, s1, o);
        pq_mma<CB>(o, acc);
    }
    if (sb < s1) {
        PqOps<CB> o;
        pq_load<CB, ONEHOT, true>(L, c, sb + 8 * q, s1, o);
        pq_mma<CB>(o, acc);
    }
    // Register i of a tile holds row 4 q + i, column c.
#pragma unroll
    for (int cb = 0; cb < CB; cb++) {
        const int j = 16 * cb + c;
        if (j >= cols)
            continue;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int r = 16 * w + 4 * q + i;
            if (r < jb.n_out)
                dst[r * cols + j] = acc[cb][i];
        }
    }
}

__global__ __launch_bounds__(kPwThreads) void paper_wgrad_bf16_kernel(PWJobs jobs,
                                                                      const __bf16 *__restrict__ qp,
                                                                      const uint16_t *__restrict__ fid,
                                                                      int64_t n,
                                                                      float *__restrict__ partial)
{
    const PWJob jb = jobs.j[blockIdx.y];
    const int cols = pw_cols(jb);
    const int lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
    const int w = threadIdx.x >> 6;
    if (16 * w >= jb.n_out)
        return;
    const int cb_n = (cols + 15) >> 4;
    const int row = 16 * w + c;
    PqLane L;
    L.qp = qp;
    L.a = row < jb.n_out ? jb.delta + row : -1;
    L.fid = fid;
    L.b_plane = false;
    L.b_const = (__bf16)0.0f;
#pragma unroll
    for (int cb = 0; cb < kPwColBlocks; cb++) {
        const int j = 16 * cb + c;
        // A column that is no plane reads the first input plane and takes its
        // constant instead.
        int plane = jb.inA;
        if (j < jb.nA)
            plane = jb.inA + j;
        else if (j < jb.nA + jb.nB)
            plane = jb.inB + j - jb.nA;
        L.b[cb] = plane;
        if (cb == cb_n - 1) {
            L.b_plane = j < jb.nA + jb.nB;
            L.b_const = (__bf16)(j < cols ? 1.0f : 0.0f);     // the bias column, or padding
        }
    }
    const int64_t s0 = (int64_t)blockIdx.x * kPwChunk;
    const int64_t s1 = s0 + kPwChunk < n ? s0 + kPwChunk : n;
    float *dst = partial + jobs.poff[blockIdx.y] + (int64_t)blockIdx.x * jb.n_out * cols;
    if (jb.onehot) {
        switch (cb_n) {
        case 1: pq_chunk<1, true>(L, jb, cols, w, q, c, s0, s1, dst); break;
        case 2: pq_chunk<2, true>(L, jb, cols, w, q, c, s0, s1, dst); break;
        case 3: pq_chunk<3, true>(L, jb, cols, w, q, c, s0, s1, dst); break;
        default: pq_chunk<4, true>(L, jb, cols, w, q, c, s0, s1, dst); break;
        }
        return;
    }
    switch (cb_n) {
    case 1: pq_chunk<1, false>(L, jb, cols, w, q, c, s0, s1, dst); break;
    case 2: pq_chunk<2, false>(L, jb, cols, w, q, c, s0, s1, dst); break;
    case 3: pq_chunk<3, false>(L, jb, cols, w, q, c, s0, s1, dst); break;
    case 4: pq_chunk<4, false>(L, jb, cols, w, q, c, s0, s1, dst); break;
    default: pq_chunk<5, false>(L, jb, cols, w, q, c, s0, s1, dst); break;
    }
}

__global__ __launch_bounds__(256) void paper_wgrad_reduce_kernel(PWJobs jobs, int n_chunks,
                                                                 const float *__restrict__ partial,
                                                                 float *__restrict__ grad,
                                                                 float *__restrict__ dsum)
{
    const PWJob jb = jobs.j[blockIdx.y];
    const int cols = pw_cols(jb);
    const int E = jb.n_out * cols;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E)
        return;
    const float *src = partial + jobs.poff[blockIdx.y] + e;
    // Eight interleaved compensated sums (independent loads in flight),
    // combined in a fixed order.
    KahanSum part[8];
    int c = 0;
    // 32 loads in flight, added in the same order as the loop below
    for (; c + 32 <= n_chunks; c += 32) {
        float v[32];
#pragma unroll
        for (int k = 0; k < 32; k++)
            v[k] = src[(int64_t)(c + k) * E];
#pragma unroll
        for (int k = 0; k < 32; k++)
            part[k & 7].add(v[k]);
    }
    for (; c + 8 <= n_chunks; c += 8) {
#pragma unroll
        for (int k = 0; k < 8; k++)
            part[k].add(src[(int64_t)(c + k) * E]);
    }
    for (; c < n_chunks; c++)
        part[0].add(src[(int64_t)c * E]);
    KahanSum tot;
#pragma unroll
    for (int k = 0; k < 8; k++)
        tot.add(part[k].value());
    const float acc = tot.value();
    const int i = e / cols, j = e % cols;
    if (jb.onehot)
        dsum[j * 64 + i] = acc;
    else if (j < jb.nA + jb.nB)
        grad[jb.w_off + i * jb.row + jb.col + j] = acc;
    else
        grad[jb.b_off + i] = acc;
}

// F1's latent columns: dWF1[o][j] = sum_f D[f][o] z_f[j]; the latents:
// dz_f[j] = sum_o WF1[o][j] D[f][o] (D: per-fabric sums of F1's gradient).
__global__ __launch_bounds__(256) void paper_latent_grads_kernel(const float *__restrict__ P, const float *__restrict__ lat,
                                          const float *__restrict__ dsum, int n_fabrics,
                                          float *__restrict__ grad, float *__restrict__ glat)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < 64 * kPLat) {
        const int o = idx / kPLat, j = idx % kPLat;
        grad[kPOffWF1 + o * kPX1 + j] = ordered_dot(dsum + o, 64, lat + j, kPLat, n_fabrics);
    } else if (idx < 64 * kPLat + n_fabrics * kPLat) {
        const int k = idx - 64 * kPLat;
        const int f = k / kPLat, j = k % kPLat;
        glat[f * kPLat + j] = ordered_dot(P + kPOffWF1 + j, kPX1, dsum + f * 64, 1, 64);
    }
}

template <typename Tp> hipError_t regrow(Tp **p, size_t count)
{
    (void)hipFree(*p);
    *p = nullptr;
    return hipMalloc((void **)p, count * sizeof(Tp));
}

PWJobs make_jobs(int n_fabrics, int n_chunks, bool fused)
{
    PWJobs J;
    auto job = [](int delta, int n_out, int inA, int nA, int inB, int nB, int w_off, int row,
                  int col, int b_off) {
        return PWJob{delta, n_out, inA, nA, inB, nB, w_off, row, col, b_off, 0};
    };
    int k = 0;
    J.j[k++] = job(kPlDY, 4, kPlG, 64, 0, 0, kPOffWA5, 64, 0, kPOffBA5);
    J.j[k++] = job(kPlDG, 64, kPlRR, 64, 0, 0, kPOffWA4, 64, 0, kPOffBA4);
    J.j[k++] = job(kPlDRR, 64, kPlH, 64, 0, 0, kPOffWA3, 64, 0, kPOffBA3);
    J.j[k++] = job(kPlDH, 64, kPlX, 64, 0, 0, kPOffWA2, 64, 0, kPOffBA2);
    if (fused) {
        J.j[k++] = job(kPlDX, 64, kPlSP, 64, kPlAng, 5, kPOffWA1, kPXA1, 0, kPOffBA1);
    } else {
        // A1 sees zeros for the angular inputs; its angular columns act in F1.
        J.j[k++] = job(kPlDX, 64, kPlSP, 64, 0, 0, kPOffWA1, kPXA1, 0, kPOffBA1);
        J.j[k++] = job(kPlDT, 64, kPlAng, 5, 0, 0, kPOffWA1, kPXA1, 64, -1);
    }
    J.j[k++] = job(kPlDSP, 64, kPlT, 64, 0, 0, kPOffWF2, 64, 0, kPOffBF2);
    J.j[k++] = job(kPlDT, 64, kPlFeat, 24, 0, 0, kPOffWF1, kPX1, kPLat, kPOffBF1);
    J.j[k++] = PWJob{kPlDT, 64, 0, n_fabrics, 0, 0, 0, 0, 0, -1, 1};
    J.n_jobs = k;
    int64_t off = 0;
    for (int q = 0; q < k; q++) {
        J.poff[q] = off;
        off += (int64_t)n_chunks * J.j[q].n_out * pw_cols(J.j[q]);
    }
    return J;
}

// The paper-size network's encoder backward (latent 64): per fabric, the
// latent's gradient back through the encoder into the scratch; then every
// encoder parameter's gradient summed over the fabrics in order.
constexpr int kPEncAct = enc_act_floats<kPLat>();
static_assert(enc_param_count<kPLat>() == kPaperEncParams, "paper encoder layout");

__global__ __launch_bounds__(kEncThreads) void paper_encoder_backward_kernel(
    const float *__restrict__ Q, const float *__restrict__ inputs, const float *__restrict__ dz,
    float *__restrict__ scratch)
{
    const int f = blockIdx.x;
    encoder_backward_block<kPLat>(Q, inputs + (size_t)f * kEncIn, dz + (size_t)f * kPLat,
                                  scratch + (size_t)f * kPEncAct);
}

__global__ void paper_encoder_wgrad_kernel(const float *__restrict__ scratch, int n_fabrics,
                                           float *__restrict__ grad)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < kPaperEncParams)
        grad[e] = encoder_wgrad_entry<kPLat>(scratch, n_fabrics, e);
}

// Loss and gradient ([params | latents], into s.grad) of one batch.
hipError_t run_paper_loss_grad(PaperTrainScratch &s, const PaperTrainArgs &a, hipStream_t stream)
{
    const fabric_train_cfg &cfg = a.cfg;
    hipError_t e;
    if (!s.grad) {
        const size_t tail = std::max((size_t)kPaperTrainMaxFabrics * kPLat, (size_t)kPaperEncParams);
        if ((e = hipMalloc((void **)&s.grad, (kPNDec + tail) * sizeof(float))) != hipSuccess) return e;
        if ((e = hipMalloc((void **)&s.lat, (size_t)kPaperTrainMaxFabrics * kPLat * sizeof(float))) != hipSuccess) return e;
        if ((e = hipMalloc((void **)&s.enc_acts, (size_t)kPaperTrainMaxFabrics * kPEncAct * sizeof(float))) != hipSuccess) return e;
        if ((e = hipMalloc((void **)&s.dsum, (size_t)kPaperTrainMaxFabrics * 64 * sizeof(float))) != hipSuccess) return e;
        if ((e = hipMalloc((void **)&s.wt, (size_t)kTFloats * sizeof(float))) != hipSuccess) return e;
        if ((e = hipMalloc((void **)&s.loss, sizeof(float))) != hipSuccess) return e;
    }
    fabric_gbuffer g;
    if (a.batch) {
        g = *a.batch;
    } else {
        const int64_t n = cfg.batch;
        if (s.batch_cap < n) {
            if ((e = regrow(&s.b_fid, (size_t)n)) != hipSuccess) return e;
            if ((e = regrow(&s.b_fields, (size_t)n * 9)) != hipSuccess) return e;
            if ((e = regrow(&s.targets, (size_t)n * 4)) != hipSuccess) return e;
            s.batch_cap = n;
        }
        fabric_gbuffer_out o;
        o.n = n;
        o.fabric_id = s.b_fid;
        float *f = s.b_fields;
        const int64_t c = s.batch_cap;
        o.u = f; o.v = f + c; o.radius = f + 2 * c; o.wi_x = f + 3 * c; o.wi_y = f + 4 * c;
        o.wi_z = f + 5 * c; o.wo_x = f + 6 * c; o.wo_y = f + 7 * c; o.wo_z = f + 8 * c;
        if ((e = launch_make_batch(cfg.seed, n, a.n_fabrics, cfg.r_lo, cfg.r_hi, cfg.btdf_frac, o,
                                   stream)) != hipSuccess)
            return e;
        g.n = n; g.fabric_id = o.fabric_id; g.u = o.u; g.v = o.v; g.radius = o.radius;
        g.wi_x = o.wi_x; g.wi_y = o.wi_y; g.wi_z = o.wi_z; g.wo_x = o.wo_x; g.wo_y = o.wo_y; g.wo_z = o.wo_z;
    }
    const int64_t n = g.n;
    const float *P = a.master, *lat = a.master + kPNDec;
    float *grad = s.grad, *glat = s.grad + kPNDec;
    if (a.enc_inputs) {
        // The latents of this step from the encoder (its parameters follow the decoder's).
        if ((e = launch_encoder_forward_n(a.master + kPNDec, a.enc_inputs, a.n_fabrics, kPLat,
                                          s.lat, stream)) != hipSuccess)
            return e;
        lat = s.lat;
    }
    if (n == 0) {
        if ((e = hipMemsetAsync(s.loss, 0, sizeof(float), stream)) != hipSuccess) return e;
        return hipMemsetAsync(s.grad, 0, (size_t)paper_trained_count(a) * sizeof(float), stream);
    }
    const float *targets = a.targets;
    if (!targets) {
        if (s.batch_cap < n) {
            // A caller-supplied batch larger than any generated one: the
            // batch planes are not in use, so all three buffers may grow.
            if ((e = regrow(&s.targets, (size_t)n * 4)) != hipSuccess) return e;
            if ((e = regrow(&s.b_fid, (size_t)n)) != hipSuccess) return e;
            if ((e = regrow(&s.b_fields, (size_t)n * 9)) != hipSuccess) return e;
            s.batch_cap = n;
        }
        if ((e = launch_gt_filter(g, a.fabrics, a.n_fabrics, cfg.gt_samples, cfg.seed ^ 1ull, a.vis,
                                  nullptr, s.targets, a.err, stream)) != hipSuccess)
            return e;
        targets = s.targets;
    }
    const int64_t blocks = (n + kFbSamples - 1) / kFbSamples;
    // The planes' stride: a multiple of 64 samples, so that the weight
    // gradients read whole 32-sample groups as aligned float4s in bounds.
    const int64_t cap = (n + 63) / 64 * 64;
    if (s.cap < cap) {
        if ((e = regrow(&s.planes, (size_t)cap * kPlanes)) != hipSuccess) return e;
        if ((e = regrow(&s.loss_part, (size_t)(cap / kFbSamples))) != hipSuccess) return e;
        s.cap = cap;
    }
    const int n_chunks = (int)((n + kPwChunk - 1) / kPwChunk);
    const PWJobs jobs = make_jobs(a.n_fabrics, n_chunks, a.fused);
    const size_t need = (size_t)(jobs.poff[jobs.n_jobs - 1] +
                                 (int64_t)n_chunks * jobs.j[jobs.n_jobs - 1].n_out *
                                     pw_cols(jobs.j[jobs.n_jobs - 1]));
    if (s.partial_floats < need) {
        if ((e = regrow(&s.partial, need)) != hipSuccess) return e;
        s.partial_floats = need;
    }
    // Faults of a generated-target batch were counted by the filter.
    (void)a.err;
    int64_t loss_parts = blocks;
    if (a.cfg.prec == FABRIC_BF16) {
        if (!s.bwd_frags &&
            (e = hipMalloc(&s.bwd_frags, (size_t)kBFrags * 64 * sizeof(bf16x8))) != hipSuccess)
            return e;
        hipLaunchKernelGGL(pack_paper_bwd_kernel, dim3((kBFrags * 64 + 255) / 256), dim3(256), 0,
                           stream, P, (bf16x8 *)s.bwd_frags);
        const auto *ffr = (const bf16x8 *)a.bf16_image;
        const auto *b5 = (const f32x4 *)(ffr + kPFrags * 64);
        loss_parts = (n + 127) / 128;
        const size_t lds = (size_t)a.n_fabrics * (64 + kFabCopies * kFabConsts) * sizeof(float);
        auto launch = [&](auto kernel) {
            hipLaunchKernelGGL(kernel, dim3((unsigned)loss_parts), dim3(256), lds, stream, g,
                               a.fabrics, a.n_fabrics, a.cfold, ffr, b5,
                               (const bf16x8 *)s.bwd_frags, targets, s.planes, s.loss_part);
        };
        if (a.raw)
            a.fused ? launch(paper_fwd_bwd_bf16_kernel<true, true>)
                    : launch(paper_fwd_bwd_bf16_kernel<true, false>);
        else
            a.fused ? launch(paper_fwd_bwd_bf16_kernel<false, true>)
                    : launch(paper_fwd_bwd_bf16_kernel<false, false>);
    } else {
        hipLaunchKernelGGL(transpose_kernel, dim3((kTFloats + 255) / 256), dim3(256), 0, stream,
                           P, s.wt);
        hipLaunchKernelGGL(paper_fwd_bwd_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, g,
                           a.fabrics, a.n_fabrics, P, lat, (const float *)s.wt, targets, s.planes,
                           s.cap, a.raw ? 1 : 0, a.fused ? 1 : 0, s.loss_part);
    }
    hipLaunchKernelGGL(paper_loss_reduce_kernel, dim3(1), dim3(256), 0, stream,
                       (const float *)s.loss_part, loss_parts, 1.0f / (float)n, s.loss);
    if (a.cfg.prec == FABRIC_BF16)
        hipLaunchKernelGGL(paper_wgrad_bf16_kernel, dim3(n_chunks, jobs.n_jobs), dim3(kPwThreads), 0,
                           stream, jobs, (const __bf16 *)s.planes, g.fabric_id, n, s.partial);
    else
        hipLaunchKernelGGL(paper_wgrad_kernel, dim3(n_chunks, jobs.n_jobs), dim3(kPwThreads), 0, stream,
                           jobs, (const float *)s.planes, s.cap, g.fabric_id, n, s.partial);
    hipLaunchKernelGGL(paper_wgrad_reduce_kernel, dim3((64 * kPwMaxIn + 255) / 256, jobs.n_jobs),
                       dim3(256), 0, stream, jobs, n_chunks, (const float *)s.partial, grad, s.dsum);
    const int tot = 64 * kPLat + a.n_fabrics * kPLat;
    hipLaunchKernelGGL(paper_latent_grads_kernel, dim3((tot + 255) / 256), dim3(256), 0, stream, P,
                       lat, (const float *)s.dsum, a.n_fabrics, grad, glat);
    if (a.enc_inputs) {
        // The latents' gradient through the encoder; its parameters' gradient
        // takes the latents' place after the decoder's.
        hipLaunchKernelGGL(paper_encoder_backward_kernel, dim3(a.n_fabrics), dim3(kEncThreads), 0, stream,
                           a.master + kPNDec, a.enc_inputs, (const float *)glat, s.enc_acts);
        hipLaunchKernelGGL(paper_encoder_wgrad_kernel, dim3((kPaperEncParams + 255) / 256),
                           dim3(256), 0, stream, (const float *)s.enc_acts, a.n_fabrics, glat);
    }
    return hipGetLastError();
}

hipError_t read_paper_loss(PaperTrainScratch &s, float *out_loss, int *finite_loss,
                           hipStream_t stream)
{
    float l = 0.0f;
    hipError_t e;
    if ((e = hipMemcpyAsync(&l, s.loss, sizeof(float), hipMemcpyDeviceToHost, stream)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(stream)) != hipSuccess) return e;
    *out_loss = l;
    *finite_loss = std::isfinite(l) ? 1 : 0;
    return hipSuccess;
}

}  // namespace

void paper_train_scratch_free(PaperTrainScratch &s)
{
    (void)hipFree(s.planes);
    (void)hipFree(s.loss_part);
    (void)hipFree(s.loss);
    (void)hipFree(s.wt);
    (void)hipFree(s.bwd_frags);
    (void)hipFree(s.partial);
    (void)hipFree(s.grad);
    (void)hipFree(s.lat);
    (void)hipFree(s.enc_acts);
    (void)hipFree(s.dsum);
    (void)hipFree(s.b_fid);
    (void)hipFree(s.b_fields);
    (void)hipFree(s.targets);
    s = PaperTrainScratch();
}

hipError_t paper_loss_grad(PaperTrainScratch &s, const PaperTrainArgs &a, float *grad_out,
                           float *out_loss, hipStream_t stream)
{
    hipError_t e = run_paper_loss_grad(s, a, stream);
    if (e != hipSuccess)
        return e;
    if ((e = hipMemcpyAsync(grad_out, s.grad, (size_t)paper_trained_count(a) * sizeof(float),
                            hipMemcpyDeviceToDevice, stream)) != hipSuccess)
        return e;
    if (out_loss) {
        int fin = 0;
        return read_paper_loss(s, out_loss, &fin, stream);
    }
    return hipSuccess;
}

hipError_t paper_train_step(PaperTrainScratch &s, const PaperTrainArgs &a, float *out_loss,
                            int *updated, hipStream_t stream)
{
    *updated = 1;
    hipError_t e = run_paper_loss_grad(s, a, stream);
    if (e != hipSuccess)
        return e;
    if ((e = launch_adam(a.master, s.grad, a.adam_m, a.adam_v, paper_trained_count(a), a.cfg,
                         a.clock, s.loss, stream)) != hipSuccess)
        return e;
    // The latents of the updated encoder, for the shading image.
    if (a.enc_inputs &&
        (e = launch_encoder_forward_n(a.master + kPNDec, a.enc_inputs, a.n_fabrics, kPLat, s.lat,
                                      stream)) != hipSuccess)
        return e;
    if (out_loss)
        return read_paper_loss(s, out_loss, updated, stream);
    return hipSuccess;
}

}  // namespace fab
