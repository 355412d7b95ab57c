// Training of the fabric network (Sec. 4.2 "Loss functions", Eq. (9)-(11);
// Sec. 5.2) with hand-written forward and backward kernels:
//
//   fwd_bwd_kernel     one 16-sample tile per wavefront: the MFMA forward of
//                      the decoder (same code as shading), the loss terms and
//                      dL/dy, then the backward through the activations as
//                      MFMA tiles with transposed weight fragments, chained in
//                      registers exactly like the forward.  Activations and
//                      activation gradients go to per-sample FP32 rows, or in
//                      BF16 training to BF16 planes blocked by 64 samples.
//   wgrad_kernel       weight gradients dW = sum_n dh_n x_n^T of every layer in
//                      one launch: FP32 MFMA tiles with samples as K, operands
//                      read straight from the per-sample rows, fixed-order
//                      reductions of the partials (deterministic).
//   wgrad_bf16_kernel  the same from the BF16 planes on BF16 MFMA 16x16x32
//                      (eight consecutive samples per lane and operand).
//   encoder kernels    per-fabric backward through the encoder and its weight
//                      gradients summed over fabrics in order.
//   adam_kernel        Adam with FP64 moments on FP32 masters; skipped on the
//                      device when the loss is not finite.
#include <cmath>
#include <cstring>

#include "enc_dense.hpp"
#include "kernels.hpp"
#include "mlp_tile.hpp"
#include "train.hpp"

namespace fab {

namespace {

// Per-sample buffer layout (floats, sample-major rows).
constexpr int kS = 40, kH1 = 64, kX3 = 72, kH3 = 64, kDY = 4, kDH = 64;
constexpr int kActFloats = kS + kH1 + kX3 + kH3 + kDY + 3 * kDH;   // 436
struct ActPtrs {
    float *S, *H1, *X3, *H3, *DY, *DH1, *DH2, *DH3;
};
__host__ __device__ inline ActPtrs act_ptrs(float *base, int64_t cap)
{
    ActPtrs a;
    a.S = base;
    a.H1 = a.S + cap * kS;
    a.X3 = a.H1 + cap * kH1;
    a.H3 = a.X3 + cap * kX3;
    a.DY = a.H3 + cap * kH3;
    a.DH1 = a.DY + cap * kDY;
    a.DH2 = a.DH1 + cap * kDH;
    a.DH3 = a.DH2 + cap * kDH;
    return a;
}

// BF16 training keeps the same quantities as planes of 16-bit values in
// the same buffer: every MFMA operand as the forward used it (features,
// activations, the angular inputs, dy) and the activation gradients rounded
// to BF16.  Blocked by 64 samples: the 433 planes of samples 64 b .. 64 b + 63
// form one contiguous region, each plane's 64 samples in order, so a lane of
// the weight gradients reads eight consecutive samples of a plane with one
// load and a block's accesses stay within 55 KB (DRAM pages are reused when
// the planes do not fit in the caches).
constexpr int kQS = 0, kQH1 = kQS + kS, kQX3 = kQH1 + kH1, kQH3 = kQX3 + 69, kQDY = kQH3 + kH3;
constexpr int kQDH1 = kQDY + kDY, kQDH2 = kQDH1 + kDH, kQDH3 = kQDH2 + kDH;
constexpr int kQPlanes = kQDH3 + kDH;                                  // 433
constexpr int kQBlock = 64;                                            // samples per region (a shift of 6)
static_assert(kQPlanes * 2 <= kActFloats * 4, "the BF16 planes fit the activation buffer");
__host__ __device__ inline int64_t q_elem(int plane, int64_t s)
{
    // s >= 0: the shift and the mask are the quotient and the remainder.
    return (s >> 6) * (kQPlanes * kQBlock) + plane * kQBlock + (s & (kQBlock - 1));
}

// Per-fabric encoder scratch (floats).
constexpr int kEncActFloats = enc_act_floats<kLatent>();
static_assert(enc_param_count<kLatent>() == kNEnc, "encoder layout");

// ---------------------------------------------------------------------------
// Training batches
// ---------------------------------------------------------------------------

__global__ void make_batch_kernel(uint64_t seed, int64_t n, int n_fabrics, float log_lo,
                                  float log_span, float btdf_frac, fabric_gbuffer_out out)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n)
        return;
    const uint64_t base = 8ull * (uint64_t)q;
    const uint64_t z0 = splitmix64_at(seed, base + 0);
    const uint64_t z1 = splitmix64_at(seed, base + 1);
    const uint64_t z2 = splitmix64_at(seed, base + 2);
    const uint64_t z3 = splitmix64_at(seed, base + 3);
    const uint64_t z4 = splitmix64_at(seed, base + 4);
    out.fabric_id[q] = (uint16_t)((uint32_t)(z0 >> 32) % (uint32_t)n_fabrics);
    out.u[q] = 8.0f * u24_hi(z1);
    out.v[q] = 8.0f * u24_mid(z1);
    out.radius[q] = expf(fmaf(u24_hi(z2), log_span, log_lo));
    float s, c, xi;
    xi = u24_hi(z3);
    sincospif(2.0f * u24_mid(z3), &s, &c);
    out.wi_x[q] = sqrtf(xi) * c;
    out.wi_y[q] = sqrtf(xi) * s;
    // Output 8q+5 lights the sample from below with probability btdf_frac.
    const float wz = sqrtf(1.0f - xi);
    out.wi_z[q] = u24_hi(splitmix64_at(seed, base + 5)) < btdf_frac ? -wz : wz;
    xi = u24_hi(z4);
    sincospif(2.0f * u24_mid(z4), &s, &c);
    out.wo_x[q] = sqrtf(xi) * c;
    out.wo_y[q] = sqrtf(xi) * s;
    out.wo_z[q] = sqrtf(1.0f - xi);
}

// ---------------------------------------------------------------------------
// Transposed weight fragments for the backward pass.
//   BW4: dh3 = W4^T dy      A[m = h3 neuron][slot] = W4[dy index][m]
//   BW3: dh2 = W3[:, :64]^T dh3   A[m = h2 neuron][slot c] = W3[chain(c)][m]
//   BW2: dh1 = W2^T dh2     A[m = h1 neuron][slot c] = W2[chain(c)][m]
// dy slots: with one K value per lane (FP32) lane group g carries dy[g];
// with eight (BF16) lane group 0 carries dy[0..3] in positions 0..3.
// ---------------------------------------------------------------------------
template <int KPL> struct BwdShape {
    static constexpr int KS2 = div_up(kChainSlots, KPL);
    static constexpr int FRAG_W4 = 0;                 // 4 M-blocks x 1 k-step
    static constexpr int FRAG_W3 = 4;                 // 4 x KS2
    static constexpr int FRAG_W2 = 4 + 4 * KS2;       // 4 x KS2
    static constexpr int NFRAG = 4 + 8 * KS2;
};

__host__ __device__ inline int dy_index(int KPL, int grp, int c)
{
    if (KPL == 1)
        return c == 0 ? grp : -1;
    return (grp == 0 && c < 4) ? c : -1;
}

template <int P>
__global__ void pack_backward_kernel(const float *__restrict__ params,
                                     typename Mfma<P>::Frag *__restrict__ frags)
{
    using M = Mfma<P>;
    using B = BwdShape<M::KPL>;
    constexpr int KPL = M::KPL;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B::NFRAG * 64)
        return;
    const int fr = idx / 64, lane = idx % 64, row = lane & 15, grp = lane >> 4;
    typename M::Frag f = M::zero();
    for (int j = 0; j < KPL; j++) {
        float w = 0.0f;
        if (fr < B::FRAG_W3) {
            const int mb = fr, m = 16 * mb + row;
            const int d = dy_index(KPL, grp, j);
            if (d >= 0) w = params[kOffW4 + d * 64 + m];
        } else if (fr < B::FRAG_W2) {
            const int mb = (fr - B::FRAG_W3) / B::KS2, ks = (fr - B::FRAG_W3) % B::KS2;
            const int m = 16 * mb + row, c = ks * KPL + j;
            if (c < kChainSlots) w = params[kOffW3 + chain_neuron(grp, c) * 69 + m];
        } else {
            const int mb = (fr - B::FRAG_W2) / B::KS2, ks = (fr - B::FRAG_W2) % B::KS2;
            const int m = 16 * mb + row, c = ks * KPL + j;
            if (c < kChainSlots) w = params[kOffW2 + chain_neuron(grp, c) * 64 + m];
        }
        M::set(f, j, w);
    }
    frags[idx] = f;
}

// ---------------------------------------------------------------------------
// Fused forward, loss and activation backward: one 16-sample tile per wave.
// GIVEN_DY: dy comes from the caller (dL/dy4 [4][n]); otherwise from the loss
// of Eq. (9)-(11) against targets [4][n] (C_warp, C_weft, S_warp, S_weft).
// max(x, 0) as the integer maximum of the bit pattern (a negative float is a
// negative integer): one instruction, where fmaxf on an MFMA result also
// quiets a signalling NaN first.
__device__ inline float relu_bits(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

// ---------------------------------------------------------------------------
// The inputs of this lane's sample of 16-sample tile `tile` (p clamped into
// the batch): its G-buffer fields and, in lane group 0, its four targets (or
// given dL/dy).
struct TileSample {
    int fid;
    float u, v, r;
    float3 wi, wo;
    float t[4];
};
__device__ inline TileSample load_tile_sample(const fabric_gbuffer &g,
                                              const float *__restrict__ tgt_or_dy, int64_t tile)
{
    const int lane = threadIdx.x & 63, grp = lane >> 4, col = lane & 15;
    const int64_t n = g.n;
    const int64_t p = tile * 16 + col;
    const int64_t pc = p < n ? p : n - 1;
    TileSample sm;
    sm.fid = g.fabric_id[pc];
    sm.u = g.u[pc];
    sm.v = g.v[pc];
    sm.r = g.radius[pc];
    sm.wi = make_float3(g.wi_x[pc], g.wi_y[pc], g.wi_z[pc]);
    sm.wo = make_float3(g.wo_x[pc], g.wo_y[pc], g.wo_z[pc]);
#pragma unroll
    for (int c = 0; c < 4; c++)
        sm.t[c] = grp == 0 ? tgt_or_dy[c * n + pc] : 0.0f;
    return sm;
}

// The forward, loss and activation backward of 16-sample tile `tile`, one
// wave (`pre`: its inputs loaded ahead by the caller, else loaded here): the per-sample results go to sink(p, valid, live, s1, a1, a2, a3,
// d1, d2, d3, dy, wi, wo) (p past the batch: valid = false, the values of a
// clamped sample with no loss and zero gradients).
// With LDSW, the forward's L2 and L3 fragments and all backward fragments
// come from `lw` (a copy in LDS: the L2 and L3 fragments, then the backward
// ones, [fragment][lane]) instead of the packed images in global memory.
template <int P, bool GIVEN_DY, typename Sink, bool LDSW = false>
__device__ inline float fwd_bwd_tile(
    const fabric_gbuffer &g, const DevFabric *__restrict__ fabrics, int n_fabrics,
    const float *__restrict__ cfold, const typename Mfma<P>::Frag *__restrict__ ffr,
    const f32x4 *__restrict__ fbias, const typename Mfma<P>::Frag *__restrict__ bfr,
    const float *__restrict__ tgt_or_dy, int64_t tile, float *__restrict__ loss_part,
    unsigned long long *err, Sink &&sink, const typename Mfma<P>::Frag *lw = nullptr,
    const TileSample *pre = nullptr)
{
    using T = Tile<P>;
    using M = typename T::M;
    using Frag = typename T::Frag;
    using B = BwdShape<T::KPL>;
    constexpr int KPL = T::KPL;

    const int lane = threadIdx.x & 63, grp = lane >> 4, col = lane & 15;
    const int64_t n = g.n;
    const int64_t p = tile * 16 + col;
    const bool valid = p < n;
    const TileSample sm = pre ? *pre : load_tile_sample(g, tgt_or_dy, tile);
    int fid = sm.fid;
    float u = sm.u, v = sm.v, r = sm.r;
    float3 wi = sm.wi, wo = sm.wo;
    const bool fault = pixel_fault(fid, n_fabrics, u, v, r, wi, wo);
    if (fault) {
        fid = 0;
        u = v = 0.0f;
        r = 1.0f;
        wi = wo = make_float3(0.0f, 0.0f, 1.0f);
    }
    const bool live = valid && !fault;
    const DevFabric &fab = fabrics[fid];
    {
        const unsigned long long bad = __ballot(grp == 0 && valid && fault);
        if (lane == 0 && bad && err)
            atomicAdd(err, (unsigned long long)__popcll(bad));
    }

    float s1[T::NS1];
    T::spatial_slots(u, v, r, fab.fwx, fab.fwy, fab.inv_wx, fab.inv_wy, grp, s1);
    f32x4 cf[4];
#pragma unroll
    for (int mb = 0; mb < 4; mb++)
        cf[mb] = *(const f32x4 *)(cfold + fid * 64 + 16 * mb + 4 * grp);
    float ang0, ang1;
    angular_slots(grp, wi, wo, &ang0, &ang1);
    using DS = DecShape<T::KPL>;
    auto getA = [&](int q) {
        if (LDSW && q >= DS::FRAG_L2 && q < DS::FRAG_L4)
            return lw[(q - DS::FRAG_L2) * 64 + lane];
        return ffr[q * 64 + lane];
    };
    auto getBias = [&](int q) { return fbias[q * 64 + lane]; };
    f32x4 a1[4], a2[4], a3[4], y;
    T::forward(getA, getBias, cf, s1, ang0, ang1, a1, a2, a3, y);

    // ---- dL/dy (lane group 0 holds y of its pixel) ----
    float dy[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    float loss = 0.0f;
    if (grp == 0 && live) {
        if (GIVEN_DY) {
#pragma unroll
            for (int c = 0; c < 4; c++)
                dy[c] = sm.t[c];
        } else {
            const float inv_n = 1.0f / (float)n;
            // g(x) = ln(k x + 1): k = 100 for reflection, 1000 for transmission.
            const float k = wi.z < 0.0f ? 10.0f * kSpec : kSpec;
#pragma unroll
            for (int c = 0; c < 4; c++) {
                const float t = sm.t[c];
                const float target = c < 2 ? t : log1pf(k * t);
                const float lam = c < 2 ? 0.1f : 0.4f;                // lambda_C, lambda_S
                const float d = y[c] - target;
                loss = fmaf(lam * d, d, loss);
                dy[c] = 2.0f * lam * d * inv_n;
            }
        }
    }
    if (!GIVEN_DY) {
        // Fixed-order sum of the 16 samples' terms (in lanes 0..15); lane 0
        // stores the tile's part unless the caller sums the tiles itself.
        for (int off = 8; off > 0; off >>= 1)
            loss += __shfl_xor(loss, off, 64);
        if (loss_part && lane == 0)
            loss_part[tile] = loss;
    }
    // Every lane fetches its pixel's dy from lane group 0.
    float dyp[4];
#pragma unroll
    for (int c = 0; c < 4; c++)
        dyp[c] = __shfl(dy[c], col, 64);

    // ---- dh3 = (W4^T dy) * [a3 > 0] ----
    Frag Bdy[1];
#pragma unroll
    for (int j = 0; j < KPL; j++) {
        const int d = dy_index(KPL, grp, j);
        float val = 0.0f;
#pragma unroll
        for (int c = 0; c < 4; c++)
            val = d == c ? dyp[c] : val;
        M::set(Bdy[0], j, val);
    }
    auto getW = [&](int q) {
        if (LDSW)
            return lw[(DS::FRAG_L4 - DS::FRAG_L2 + q) * 64 + lane];
        return bfr[q * 64 + lane];
    };
    f32x4 d3[4], d2[4], d1[4];
#pragma unroll
    for (int mb = 0; mb < 4; mb++)
        d3[mb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    T::template dense<4>(getW, B::FRAG_W4, Bdy, d3);
#pragma unroll
    for (int mb = 0; mb < 4; mb++)
#pragma unroll
        for (int i = 0; i < 4; i++)
            d3[mb][i] = a3[mb][i] > 0.0f ? d3[mb][i] : 0.0f;

    // ---- dh2 = (W3[:, :64]^T dh3) * [a2 > 0] ----
    Frag Bd3[B::KS2];
    T::chain(d3, false, Bd3);
#pragma unroll
    for (int mb = 0; mb < 4; mb++)
        d2[mb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    T::template dense<4>(getW, B::FRAG_W3, Bd3, d2);
#pragma unroll
    for (int mb = 0; mb < 4; mb++)
#pragma unroll
        for (int i = 0; i < 4; i++)
            d2[mb][i] = a2[mb][i] > 0.0f ? d2[mb][i] : 0.0f;

    // ---- dh1 = (W2^T dh2) * [a1 > 0] ----
    Frag Bd2[B::KS2];
    T::chain(d2, false, Bd2);
#pragma unroll
    for (int mb = 0; mb < 4; mb++)
        d1[mb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    T::template dense<4>(getW, B::FRAG_W2, Bd2, d1);
#pragma unroll
    for (int mb = 0; mb < 4; mb++)
#pragma unroll
        for (int i = 0; i < 4; i++)
            d1[mb][i] = a1[mb][i] > 0.0f ? d1[mb][i] : 0.0f;

    sink(p, valid, live, s1, a1, a2, a3, d1, d2, d3, dy, wi, wo);
    return loss;
}

// Fused forward, loss and activation backward: one 16-sample tile per wave;
// the activations and activation gradients go to per-sample FP32 rows, or
// in BF16 training to BF16 planes blocked by 64 samples.
template <int P, bool GIVEN_DY>
__global__ __launch_bounds__(256) void fwd_bwd_kernel(
    fabric_gbuffer g, const DevFabric *__restrict__ fabrics, int n_fabrics,
    const float *__restrict__ cfold, const typename Mfma<P>::Frag *__restrict__ ffr,
    const f32x4 *__restrict__ fbias, const typename Mfma<P>::Frag *__restrict__ bfr,
    const float *__restrict__ tgt_or_dy, float *__restrict__ acts, int64_t cap,
    float *__restrict__ loss_part, unsigned long long *err)
{
    using T = Tile<P>;
    // BF16 training writes the blocked BF16 planes (see kQPlanes).
    constexpr bool kQ = P == FABRIC_BF16 && !GIVEN_DY;
    const int grp = (threadIdx.x & 63) >> 4;
    const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile * 16 >= g.n)      // whole wave past the end (last block)
        return;
    auto sink = [&](int64_t p, bool valid, bool live, const float (&s1)[T::NS1],
                    const f32x4 (&a1)[4], const f32x4 (&a2)[4], const f32x4 (&a3)[4],
                    const f32x4 (&d1)[4], const f32x4 (&d2)[4], const f32x4 (&d3)[4],
                    const float (&dy)[4], float3 wi, float3 wo) {
        if (!valid)
            return;
        const float keep = live ? 1.0f : 0.0f;
        if (kQ) {
            // ---- per-sample BF16 planes for the weight gradients ----
            __bf16 *qp = (__bf16 *)acts;
            auto put = [&](int plane, float x) { qp[q_elem(plane, p)] = (__bf16)x; };
#pragma unroll
            for (int c = 0; c < kL1Slots; c++)
                put(kQS + l1_feature(grp, c), s1[c]);
#pragma unroll
            for (int mb = 0; mb < 4; mb++) {
                const int o = 16 * mb + 4 * grp;
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    put(kQH1 + o + i, relu_bits(a1[mb][i]));
                    put(kQX3 + o + i, relu_bits(a2[mb][i]));
                    put(kQH3 + o + i, relu_bits(a3[mb][i]));
                    put(kQDH1 + o + i, d1[mb][i] * keep);
                    put(kQDH2 + o + i, d2[mb][i] * keep);
                    put(kQDH3 + o + i, d3[mb][i] * keep);
                }
            }
            if (grp == 0) {
                put(kQX3 + 64, wi.x);
                put(kQX3 + 65, wi.y);
                put(kQX3 + 66, wi.z);
                put(kQX3 + 67, wo.x);
                put(kQX3 + 68, wo.y);
#pragma unroll
                for (int c = 0; c < 4; c++)
                    put(kQDY + c, dy[c]);
            }
            return;
        }
        // ---- per-sample rows for the weight gradients ----
        ActPtrs ap = act_ptrs(acts, cap);
#pragma unroll
        for (int c = 0; c < kL1Slots; c++)
            ap.S[p * kS + l1_feature(grp, c)] = s1[c];
#pragma unroll
        for (int mb = 0; mb < 4; mb++) {
            const int o = 16 * mb + 4 * grp;
            f32x4 h1, h2, h3;
#pragma unroll
            for (int i = 0; i < 4; i++) {
                h1[i] = relu_bits(a1[mb][i]);
                h2[i] = relu_bits(a2[mb][i]);
                h3[i] = relu_bits(a3[mb][i]);
            }
            *(f32x4 *)(ap.H1 + p * kH1 + o) = h1;
            *(f32x4 *)(ap.X3 + p * kX3 + o) = h2;
            *(f32x4 *)(ap.H3 + p * kH3 + o) = h3;
            *(f32x4 *)(ap.DH1 + p * kDH + o) = d1[mb] * keep;
            *(f32x4 *)(ap.DH2 + p * kDH + o) = d2[mb] * keep;
            *(f32x4 *)(ap.DH3 + p * kDH + o) = d3[mb] * keep;
        }
        if (grp == 0) {
            float *x3 = ap.X3 + p * kX3;
            x3[64] = wi.x;
            x3[65] = wi.y;
            x3[66] = wi.z;
            x3[67] = wo.x;
            x3[68] = wo.y;
            x3[69] = 0.0f;
            x3[70] = 0.0f;
            x3[71] = 0.0f;
            *(f32x4 *)(ap.DY + p * kDY) = f32x4{dy[0], dy[1], dy[2], dy[3]};
        }
    };
    fwd_bwd_tile<P, GIVEN_DY>(g, fabrics, n_fabrics, cfold, ffr, fbias, bfr, tgt_or_dy, tile,
                              loss_part, err, sink);
}

// ---------------------------------------------------------------------------
// Weight gradients as sums of outer products over samples, all jobs of a
// step in one launch: job j computes
//   out_j[m][c] = sum_s A_j[s][m] * Bx_j[s][c],   m < MA <= 64, c < NC <= 80,
// where Bx is B's first NB columns followed (with a bias) by a column of
// ones, or (ids != NULL) the one-hot of ids over fabrics f0 .. f0+NC-1.
// Samples are the K dimension of FP32 MFMA 16x16x4 tiles whose operands are
// read straight from the sample-major rows: lane l takes sample 4k + l/16 and
// column l%16 of a 16-wide slab, which are 16 consecutive floats of a row.
// Every wave keeps all (up to 4 x 5) output tiles of its job in registers
// over its share of the samples; the block's four waves are summed through
// LDS in wave order, and the blocks' partials by wgrad_reduce_kernel in block
// order, so the result is deterministic.
// ---------------------------------------------------------------------------
constexpr int kWgMaxM = 64, kWgMaxC = 80;
constexpr int kWgMT = kWgMaxM / 16, kWgCT = kWgMaxC / 16;
constexpr int kWgBlocks = 128;   // partial sums per job
constexpr int kWgMaxJobs = 8;

struct WgJob {
    const float *A;           // [n][lda], columns 0..MA-1 used
    const float *B;           // [n][ldb], columns 0..NB-1 used (NULL with ids)
    const uint16_t *ids;      // one-hot source, or NULL
    int lda, MA, ldb, NB, bias, f0, NC;
};
struct WgJobs {
    WgJob j[kWgMaxJobs];
};

__global__ __launch_bounds__(256) void wgrad_kernel(WgJobs jobs, int64_t n, int64_t per_block,
                                                    float *__restrict__ partial)
{
    __shared__ float red[4][kWgMaxM * kWgMaxC / 4];   // one quarter of the tile per pass
    const WgJob jb = jobs.j[blockIdx.y];
    const int lane = threadIdx.x & 63, grp = lane >> 4, col = lane & 15;
    const int wave = threadIdx.x >> 6;
    const int MT = (jb.MA + 15) >> 4, CT = (jb.NC + 15) >> 4;
    const int64_t b0 = (int64_t)blockIdx.x * per_block;
    const int64_t b1 = b0 + per_block < n ? b0 + per_block : n;
    // The block's samples are dealt to its waves in runs of 16 (four k-steps).
    f32x4 acc[kWgMT][kWgCT];
#pragma unroll
    for (int mt = 0; mt < kWgMT; mt++)
#pragma unroll
        for (int ct = 0; ct < kWgCT; ct++)
            acc[mt][ct] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int64_t base = b0 + 16 * wave; base < b1; base += 64) {
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int64_t smp = base + 4 * k + grp;
            const bool in = smp < b1;
            float av[kWgMT], bv[kWgCT];
#pragma unroll
            for (int mt = 0; mt < kWgMT; mt++) {
                const int m = 16 * mt + col;
                av[mt] = (in && mt < MT && m < jb.MA) ? jb.A[smp * jb.lda + m] : 0.0f;
            }
            const int fid = (in && jb.ids) ? (int)jb.ids[smp] : -1;
#pragma unroll
            for (int ct = 0; ct < kWgCT; ct++) {
                const int c = 16 * ct + col;
                float v = 0.0f;
                if (in && ct < CT && c < jb.NC) {
                    if (jb.ids)
                        v = fid == jb.f0 + c ? 1.0f : 0.0f;
                    else if (c < jb.NB)
                        v = jb.B[smp * jb.ldb + c];
                    else
                        v = jb.bias ? 1.0f : 0.0f;
                }
                bv[ct] = v;
            }
#pragma unroll
            for (int mt = 0; mt < kWgMT; mt++)
#pragma unroll
                for (int ct = 0; ct < kWgCT; ct++)
                    if (mt < MT && ct < CT)
                        acc[mt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mt], bv[ct], acc[mt][ct], 0, 0, 0);
        }
    }
    // Sum the four waves' tiles in wave order, one M-tile row at a time, and
    // write the block's partial [kWgMaxM][kWgMaxC].
    float *out = partial + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * (kWgMaxM * kWgMaxC);
#pragma unroll
    for (int mt = 0; mt < kWgMT; mt++) {
        // red[w][ (m%16) * kWgMaxC + c ] for the 16 rows of M-tile mt
#pragma unroll
        for (int ct = 0; ct < kWgCT; ct++)
#pragma unroll
            for (int i = 0; i < 4; i++)
                red[wave][(4 * grp + i) * kWgMaxC + 16 * ct + col] = acc[mt][ct][i];
        __syncthreads();
        for (int e = threadIdx.x; e < 16 * kWgMaxC; e += blockDim.x) {
            const float v = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
            out[(16 * mt) * kWgMaxC + e] = v;
        }
        __syncthreads();
    }
}

// BF16 training's weight gradients, from the blocked BF16 planes: the same jobs and
// partial layout as wgrad_kernel, on BF16 MFMA 16x16x32 with samples as K.
// Wave w of a block takes the job's output rows 16 w .. 16 w + 15 for every
// 16-column block over the block's samples; lane (q = l/16, c = l%16) holds
// samples s + 8 q .. s + 8 q + 7 of its row's delta plane and of its
// column's input plane (one 16-byte load each), which fill k slots 8 q .. 8 q
// + 7 of both operands alike.  A job's column blocks but the last hold input
// planes only; the last mixes planes, the bias column (1) and padding (0);
// the one-hot job compares fabric ids.  Samples past the batch enter as
// zeros in both operands.  The waves' rows are disjoint: no block sum.
struct WgJob16 {
    int A;                    // first delta plane, rows 0..MA-1
    int B;                    // first input plane, columns 0..NB-1 (-1 with ids)
    const uint16_t *ids;
    int MA, NB, bias, f0, NC;
};
struct WgJobs16 {
    WgJob16 j[kWgMaxJobs];
};
constexpr int kWg16ColBlocks = kWgMaxC / 16;

struct Wg16Lane {
    const __bf16 *qp;                 // the planes
    int a;                            // the lane's delta plane (-1: a padding row)
    int b[kWg16ColBlocks];            // the lane's column planes
    bool b_plane;                     // the last block's column is a plane
    __bf16 b_const;                   // else its value
    const uint16_t *ids;
    int f0, NC;
};

template <int CB> struct Wg16Ops {
    bf16x8 a;
    bf16x8 b[CB];
};

template <int CB, bool ONEHOT, bool TAIL>
__device__ inline void wg16_load(const Wg16Lane &L, int c, int64_t base, int64_t s1, Wg16Ops<CB> &o)
{
    const __bf16 zero = (__bf16)0.0f, one = (__bf16)1.0f;
    auto in = [&](int t) { return !TAIL || base + t < s1; };
    // base is a multiple of 8: the eight samples lie in one region.
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
            id[t] = in(t) ? (int)L.ids[base + t] - L.f0 : -1;
#pragma unroll
        for (int cb = 0; cb < CB; cb++) {
            const int j = 16 * cb + c;
#pragma unroll
            for (int t = 0; t < 8; t++)
                o.b[cb][t] = j < L.NC && id[t] == j ? one : zero;
        }
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
__device__ inline void wg16_mma(const Wg16Ops<CB> &o, f32x4 (&acc)[CB])
{
#pragma unroll
    for (int cb = 0; cb < CB; cb++)
        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(o.a, o.b[cb], acc[cb], 0, 0, 0);
}

template <int CB, bool ONEHOT>
__device__ inline void wg16_block(const Wg16Lane &L, int MA, int NC, int w, int q, int c,
                                  int64_t s0, int64_t s1, float *__restrict__ out)
{
    f32x4 acc[CB];
#pragma unroll
    for (int cb = 0; cb < CB; cb++)
        acc[cb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    int64_t sb = s0;
    for (; sb + 32 <= s1; sb += 32) {
        Wg16Ops<CB> o;
        wg16_load<CB, ONEHOT, false>(L, c, sb + 8 * q, s1, o);
        wg16_mma<CB>(o, acc);
    }
    if (sb < s1) {
        Wg16Ops<CB> o;
        wg16_load<CB, ONEHOT, true>(L, c, sb + 8 * q, s1, o);
        wg16_mma<CB>(o, acc);
    }
    // Register i of a tile holds row 4 q + i, column c.
#pragma unroll
    for (int cb = 0; cb < CB; cb++) {
        const int j = 16 * cb + c;
        if (j >= NC)
            continue;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int m = 16 * w + 4 * q + i;
            if (m < MA)
                out[m * kWgMaxC + j] = acc[cb][i];
        }
    }
}

__global__ __launch_bounds__(256) void wgrad_bf16_kernel(WgJobs16 jobs, int64_t n,
                                                         const __bf16 *__restrict__ qp,
                                                         int64_t per_block,
                                                         float *__restrict__ partial)
{
    const WgJob16 jb = jobs.j[blockIdx.y];
    const int lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
    const int w = threadIdx.x >> 6;
    if (16 * w >= jb.MA)
        return;
    const int row = 16 * w + c;
    Wg16Lane L;
    L.qp = qp;
    L.a = row < jb.MA ? jb.A + row : -1;
    L.ids = jb.ids;
    L.f0 = jb.f0;
    L.NC = jb.NC;
    L.b_plane = false;
    L.b_const = (__bf16)0.0f;
    const int cb_n = (jb.NC + 15) >> 4;
#pragma unroll
    for (int cb = 0; cb < kWg16ColBlocks; cb++) {
        const int j = 16 * cb + c;
        // A column that is no plane reads the first input plane (in bounds)
        // and takes its constant instead.
        L.b[cb] = jb.B >= 0 ? jb.B + (j < jb.NB ? j : 0) : 0;
        if (cb == cb_n - 1) {
            L.b_plane = j < jb.NB;
            L.b_const = (__bf16)(j < jb.NC && jb.bias ? 1.0f : 0.0f);
        }
    }
    const int64_t s0 = (int64_t)blockIdx.x * per_block;
    const int64_t s1 = s0 + per_block < n ? s0 + per_block : n;
    float *out = partial + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * (kWgMaxM * kWgMaxC);
    if (jb.ids) {
        switch (cb_n) {
        case 1: wg16_block<1, true>(L, jb.MA, jb.NC, w, q, c, s0, s1, out); break;
        case 2: wg16_block<2, true>(L, jb.MA, jb.NC, w, q, c, s0, s1, out); break;
        case 3: wg16_block<3, true>(L, jb.MA, jb.NC, w, q, c, s0, s1, out); break;
        default: wg16_block<4, true>(L, jb.MA, jb.NC, w, q, c, s0, s1, out); break;
        }
        return;
    }
    switch (cb_n) {
    case 1: wg16_block<1, false>(L, jb.MA, jb.NC, w, q, c, s0, s1, out); break;
    case 2: wg16_block<2, false>(L, jb.MA, jb.NC, w, q, c, s0, s1, out); break;
    case 3: wg16_block<3, false>(L, jb.MA, jb.NC, w, q, c, s0, s1, out); break;
    case 4: wg16_block<4, false>(L, jb.MA, jb.NC, w, q, c, s0, s1, out); break;
    default: wg16_block<5, false>(L, jb.MA, jb.NC, w, q, c, s0, s1, out); break;
    }
}

// ---------------------------------------------------------------------------
// BF16 training in one persistent kernel, the activations kept on chip: a
// block of kFWaves waves takes kFChunk consecutive samples at a time; each
// wave runs the forward, loss and activation backward of its 16 samples
// (fwd_bwd_tile) and writes the per-sample values - every MFMA operand as
// the forward used it and the activation gradients, rounded to BF16 - as
// rows of the block's LDS region ([plane][sample], the planes of kQPlanes);
// after a barrier the waves accumulate the weight gradients of those
// samples from the region on BF16 MFMA 16x16x32 (samples as K: lane
// (q = l/16, c = l%16) reads samples 8q .. 8q + 7 of a 32-sample step from
// row c of the tile's delta planes and of its input planes, one 16-byte read
// each), a wave owning the tiles w, w + kFWaves, ... of the step's 16x16
// output tiles over all its chunks; a second barrier frees the region for
// the next chunk.  The tiles' sums go to the partial layout of
// wgrad_kernel (one partial per block), summed by wgrad_reduce_kernel.
// Samples past the batch run on a clamped sample with zero gradients and
// add nothing.
// ---------------------------------------------------------------------------
constexpr int kFWaves = 8;
constexpr int kFChunk = 16 * kFWaves;        // samples per chunk
constexpr int kFStride = kFChunk + 8;        // LDS row of a plane (BF16 values)
constexpr int kFMaxSlots = 8;                // output tiles per wave
constexpr int kFMaxTiles = kFMaxSlots * kFWaves;
constexpr size_t kFTileOfs = (size_t)kQPlanes * kFStride * 2 + (size_t)kFChunk * 2;
constexpr size_t kFConstOfs = kFTileOfs + (size_t)kFMaxTiles * 16;
constexpr size_t kFWOfs = kFConstOfs + (size_t)2 * kFStride * 2;
// the L2, L3 and backward fragments of the decoder image, [fragment][lane]
constexpr int kFWFrags = DecShape<8>::FRAG_L4 - DecShape<8>::FRAG_L2 + BwdShape<8>::NFRAG;
constexpr size_t kFLds = kFWOfs + (size_t)kFWFrags * 64 * 16;
static_assert(kFLds <= 160 * 1024, "the region fits in a CU's LDS");

struct FusedJobs {
    WgJob16 j[kWgMaxJobs];       // A, B: first planes of the region (B < 0: one-hot)
    int first_tile[kWgMaxJobs + 1];
    int n_jobs;
};

typedef short s16x8 __attribute__((ext_vector_type(8)));

// Output tile t of the weight gradients, in the terms of the lane (q, c)
// that accumulates rows 4q.. of column c: x = first delta plane of its rows,
// y = rows present, z = first input plane of its columns (one-hot: the fabric
// id of column 0), w = columns present (bits 0-7), one-hot (bit 8) and the
// column carrying the bias constant (bits 9-13; 31: none).  Built once per
// block from the job table, so that the chunks' loops read one LDS word per
// tile instead of searching the table.
__device__ inline int4 fused_tile_desc(const FusedJobs &jobs, int t)
{
    int jn = 0;
    while (jn + 1 < jobs.n_jobs && t >= jobs.first_tile[jn + 1])
        jn++;
    const WgJob16 jb = jobs.j[jn];
    const int nbk = (jb.NC + 15) >> 4;
    const int local = t - jobs.first_tile[jn];
    const int mb = local / nbk, nb = local % nbk;
    auto clamp16 = [](int v) { return v < 0 ? 0 : (v > 16 ? 16 : v); };
    const bool onehot = jb.B < 0;
    const int bias_col = !onehot && jb.bias ? jb.NB - 16 * nb : -1;
    int4 d;
    d.x = jb.A + 16 * mb;
    d.y = clamp16(jb.MA - 16 * mb);
    d.z = onehot ? jb.f0 + 16 * nb : jb.B + 16 * nb;
    d.w = clamp16(onehot ? jb.NC - 16 * nb : jb.NB - 16 * nb) | (onehot ? 1 << 8 : 0) |
          ((bias_col >= 0 && bias_col < 16 ? bias_col : 31) << 9);
    return d;
}

__global__ __launch_bounds__(64 * kFWaves) void train_bf16_fused_kernel(
    fabric_gbuffer g, const DevFabric *__restrict__ fabrics, int n_fabrics,
    const float *__restrict__ cfold, const bf16x8 *__restrict__ ffr,
    const f32x4 *__restrict__ fbias, const bf16x8 *__restrict__ bfr,
    const float *__restrict__ targets, float *__restrict__ loss_part, unsigned long long *err,
    FusedJobs jobs, int64_t n_chunks, float *__restrict__ partial)
{
    using T = Tile<FABRIC_BF16>;
    extern __shared__ __align__(16) unsigned char f_smem[];
    __bf16 *region = (__bf16 *)f_smem;
    uint16_t *s_fid = (uint16_t *)(f_smem + (size_t)kQPlanes * kFStride * 2);
    int4 *s_tile = (int4 *)(f_smem + kFTileOfs);
    // a row of zeros and a row of ones (BF16 1.0): the operand rows of a
    // tile's absent rows and columns and of its bias column
    __bf16 *zero_row = (__bf16 *)(f_smem + kFConstOfs), *one_row = zero_row + kFStride;
    const int lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n_tiles = jobs.first_tile[jobs.n_jobs];
    if ((int)threadIdx.x < n_tiles)
        s_tile[threadIdx.x] = fused_tile_desc(jobs, threadIdx.x);
    for (int k = threadIdx.x; k < kFStride; k += blockDim.x) {
        zero_row[k] = (__bf16)0.0f;
        one_row[k] = (__bf16)1.0f;
    }
    bf16x8 *s_w = (bf16x8 *)(f_smem + kFWOfs);
    {
        constexpr int kFwd = (DecShape<8>::FRAG_L4 - DecShape<8>::FRAG_L2) * 64;
        for (int k = threadIdx.x; k < kFWFrags * 64; k += blockDim.x)
            s_w[k] = k < kFwd ? ffr[DecShape<8>::FRAG_L2 * 64 + k] : bfr[k - kFwd];
    }
    __syncthreads();

    f32x4 acc[kFMaxSlots];
#pragma unroll
    for (int k = 0; k < kFMaxSlots; k++)
        acc[k] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    // The loss terms of the wave's tiles, summed in chunk order (lane 0).
    float wave_loss = 0.0f;

    // The samples of the wave's next tile, loaded one chunk ahead (during the
    // previous chunk's weight-gradient phase).
    TileSample next;
    if ((int64_t)blockIdx.x < n_chunks)
        next = load_tile_sample(g, targets, (int64_t)blockIdx.x * kFWaves + w);
    for (int64_t chunk = blockIdx.x; chunk < n_chunks; chunk += gridDim.x) {
        // ---- the wave's 16 samples into the region ----
        const int64_t tile = chunk * kFWaves + w;
        const TileSample cur = next;
        auto sink = [&](int64_t p, bool valid, bool live, const float (&s1)[T::NS1],
                        const f32x4 (&a1)[4], const f32x4 (&a2)[4], const f32x4 (&a3)[4],
                        const f32x4 (&d1)[4], const f32x4 (&d2)[4], const f32x4 (&d3)[4],
                        const float (&dy)[4], float3 wi, float3 wo) {
            // A sample without a loss term (past the batch or faulted) has
            // dy = 0, so its activation gradients are exact zeros already.
            (void)valid;
            (void)live;
            const int sl = 16 * w + c;
            auto put = [&](int plane, float x) { region[plane * kFStride + sl] = (__bf16)x; };
#pragma unroll
            for (int k = 0; k < kL1Slots; k++)
                put(kQS + l1_feature(q, k), s1[k]);
#pragma unroll
            for (int mb = 0; mb < 4; mb++) {
                const int o = 16 * mb + 4 * q;
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    put(kQH1 + o + i, relu_bits(a1[mb][i]));
                    put(kQX3 + o + i, relu_bits(a2[mb][i]));
                    put(kQH3 + o + i, relu_bits(a3[mb][i]));
                    put(kQDH1 + o + i, d1[mb][i]);
                    put(kQDH2 + o + i, d2[mb][i]);
                    put(kQDH3 + o + i, d3[mb][i]);
                }
            }
            if (q == 0) {
                put(kQX3 + 64, wi.x);
                put(kQX3 + 65, wi.y);
                put(kQX3 + 66, wi.z);
                put(kQX3 + 67, wo.x);
                put(kQX3 + 68, wo.y);
#pragma unroll
                for (int k = 0; k < 4; k++)
                    put(kQDY + k, dy[k]);
                s_fid[sl] = (uint16_t)g.fabric_id[p < g.n ? p : g.n - 1];
            }
        };
        // An offset the compiler cannot see through, so that the decoder's
        // weight reads stay inside the loop instead of being hoisted into
        // registers for all chunks (they would not fit beside the tiles' sums).
        int wofs = 0;
        asm volatile("" : "+s"(wofs));
        wave_loss += fwd_bwd_tile<FABRIC_BF16, false, decltype(sink) &, true>(
            g, fabrics, n_fabrics, cfold, ffr + wofs, fbias + wofs, bfr + wofs, targets, tile,
            nullptr, err, sink, s_w + wofs, &cur);
        __syncthreads();
        if (chunk + gridDim.x < n_chunks)
            next = load_tile_sample(g, targets, (chunk + gridDim.x) * kFWaves + w);

        // ---- the chunk's weight-gradient terms ----
#pragma unroll
        for (int slot = 0; slot < kFMaxSlots; slot++) {
            const int t = slot * kFWaves + w;
            if (t >= n_tiles)
                continue;
            const int4 dv = s_tile[t];
            const int a0 = __builtin_amdgcn_readfirstlane(dv.x);
            const int na = __builtin_amdgcn_readfirstlane(dv.y);
            const int b0 = __builtin_amdgcn_readfirstlane(dv.z);
            const int info = __builtin_amdgcn_readfirstlane(dv.w);
            const int nb = info & 0xff;
            const __bf16 *arow = c < na ? region + (a0 + c) * kFStride : zero_row;
            if (info & (1 << 8)) {
                // one-hot columns: fabric b0 + c
#pragma unroll
                for (int ks = 0; ks < kFChunk / 32; ks++) {
                    const int k0 = 32 * ks + 8 * q;
                    const bf16x8 a = *(const bf16x8 *)(arow + k0);
                    s16x8 b;
#pragma unroll
                    for (int j = 0; j < 8; j++)
                        b[j] = (int)s_fid[k0 + j] - b0 == c && c < nb ? (short)0x3F80 : (short)0;
                    acc[slot] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        a, __builtin_bit_cast(bf16x8, b), acc[slot], 0, 0, 0);
                }
            } else {
                const __bf16 *brow = c < nb ? region + (b0 + c) * kFStride
                                            : (c == ((info >> 9) & 31) ? one_row : zero_row);
#pragma unroll
                for (int ks = 0; ks < kFChunk / 32; ks++) {
                    const int k0 = 32 * ks + 8 * q;
                    const bf16x8 a = *(const bf16x8 *)(arow + k0);
                    const bf16x8 b = *(const bf16x8 *)(brow + k0);
                    acc[slot] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[slot], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }

    // ---- the block's loss part: its waves' sums in wave order ----
    __shared__ float s_wave_loss[kFWaves];
    if (lane == 0)
        s_wave_loss[w] = wave_loss;
    __syncthreads();
    if (threadIdx.x == 0) {
        float l = 0.0f;
        for (int k = 0; k < kFWaves; k++)
            l += s_wave_loss[k];
        loss_part[blockIdx.x] = l;
    }

    // ---- the block's partial sums: register i of a tile holds row 4 q + i, column c ----
#pragma unroll
    for (int slot = 0; slot < kFMaxSlots; slot++) {
        const int t = slot * kFWaves + w;
        if (t >= n_tiles)
            continue;
        int jn = 0;
        while (jn + 1 < jobs.n_jobs && t >= jobs.first_tile[jn + 1])
            jn++;
        const WgJob16 jb = jobs.j[jn];
        const int nbk = (jb.NC + 15) >> 4;
        const int local = t - jobs.first_tile[jn];
        const int mb = local / nbk, nb = local % nbk;
        float *out = partial + ((size_t)jn * gridDim.x + blockIdx.x) * (kWgMaxM * kWgMaxC);
        const int colj = 16 * nb + c;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int m = 16 * mb + 4 * q + i;
            if (m < jb.MA && colj < jb.NC)
                out[m * kWgMaxC + colj] = acc[slot][i];
        }
    }
}

// out_j[m][c] = sum over the blocks' partials (four consecutive ranges of
// blocks, each summed in block order as eight interleaved running sums, all
// combined in a fixed order), scattered to
// dst[m * ldw + c] (c < NW), bias[m] (c == NW with a bias), or with
// transposed = 1 to dst[c * ldw + m].
struct WgDest {
    float *dst, *bias;
    int MA, NC, NW, ldw, transposed;
};
struct WgDests {
    WgDest d[kWgMaxJobs];
};

// A block takes 64 entries; its four waves sum the partials of four
// consecutive ranges of blocks for them (eight interleaved running sums per
// range, 32 loads in flight), combined through LDS in a fixed order.
constexpr int kWgRedEntries = 64;
__global__ __launch_bounds__(256) void wgrad_reduce_kernel(const float *__restrict__ partial,
                                                           WgDests dests, int nblk)
{
    __shared__ float part[4][kWgRedEntries];
    const WgDest d = dests.d[blockIdx.y];
    const int seg = threadIdx.x >> 6;
    const int e = blockIdx.x * kWgRedEntries + (threadIdx.x & 63);
    const bool live = e < d.MA * d.NC;
    const int m = live ? e / d.NC : 0, c = live ? e % d.NC : 0;
    const int per = (nblk + 3) >> 2;
    const int b0 = seg * per, b1 = min(nblk, b0 + per);
    const float *p = partial + (size_t)blockIdx.y * nblk * (kWgMaxM * kWgMaxC) + m * kWgMaxC + c;
    float r[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    if (live) {
        int b = b0;
        for (; b + 32 <= b1; b += 32) {
            float v[32];
#pragma unroll
            for (int k = 0; k < 32; k++)
                v[k] = p[(size_t)(b + k) * (kWgMaxM * kWgMaxC)];
#pragma unroll
            for (int k = 0; k < 32; k++)
                r[k & 7] += v[k];
        }
        for (; b < b1; b++)
            r[(b - b0) & 7] += p[(size_t)b * (kWgMaxM * kWgMaxC)];
    }
    part[seg][threadIdx.x & 63] = ((r[0] + r[1]) + (r[2] + r[3])) + ((r[4] + r[5]) + (r[6] + r[7]));
    __syncthreads();
    if (seg != 0 || !live)
        return;
    const int i = threadIdx.x;
    const float acc = (part[0][i] + part[1][i]) + (part[2][i] + part[3][i]);
    if (d.transposed)
        d.dst[c * d.ldw + m] = acc;
    else if (c < d.NW)
        d.dst[m * d.ldw + c] = acc;
    else if (d.bias)
        d.bias[m] = acc;
}

// dz_f = W1[:, 0:32]^T dc_f and dW1[:, 0:32] = sum_f dc_f z_f^T.
__global__ __launch_bounds__(256) void latent_grads_kernel(const float *__restrict__ params, const float *__restrict__ dcf,
                                    const float *__restrict__ latents, int n_fabrics,
                                    float *__restrict__ dz, float *__restrict__ dW1)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n_fabrics * kLatent) {
        const int f = e / kLatent, k = e % kLatent;
        dz[e] = ordered_dot(params + kOffW1 + k, 72, dcf + f * 64, 1, 64);
    }
    if (e < 64 * kLatent) {
        const int o = e / kLatent, k = e % kLatent;
        dW1[o * 72 + k] = ordered_dot(dcf + o, 64, latents + k, kLatent, n_fabrics);
    }
}

// ---------------------------------------------------------------------------
// Encoder backward.  Per fabric: recompute the forward and backpropagate dz
// to the pre-activation gradients; then every weight gradient is a sum over
// fabrics in order.
// enc scratch per fabric: x[524] a1 a2 a3 da1 da2 da3 [128 each] dz[32]
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kEncThreads) void encoder_backward_kernel(
    const float *__restrict__ Q, const float *__restrict__ inputs, const float *__restrict__ dz,
    float *__restrict__ scratch)
{
    const int f = blockIdx.x;
    encoder_backward_block<kLatent>(Q, inputs + (size_t)f * kEncIn, dz + (size_t)f * kLatent,
                                    scratch + (size_t)f * kEncActFloats);
}

// One thread per encoder parameter: the sum over fabrics, in order.
__global__ void encoder_wgrad_kernel(const float *__restrict__ scratch, int n_fabrics,
                                     float *__restrict__ grad)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < kNEnc)
        grad[e] = encoder_wgrad_entry<kLatent>(scratch, n_fabrics, e);
}

// ---------------------------------------------------------------------------
// Loss reduction and Adam
// ---------------------------------------------------------------------------
// The batch loss: per thread a compensated sum of every 256th part, then a
// fixed tree over the threads.
__global__ __launch_bounds__(256) void loss_reduce_kernel(const float *__restrict__ part,
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

// First stage of the loss of a large batch: block b sums the parts
// [b seg, (b + 1) seg) the way loss_reduce_kernel sums its input (a
// compensated sum per thread, then a fixed tree), so the whole reduction
// keeps a fixed order.
constexpr int kLossStage = 256;     // first-stage blocks at most
__global__ __launch_bounds__(256) void loss_stage_kernel(const float *__restrict__ part,
                                                         int64_t nparts, int64_t seg,
                                                         float *__restrict__ out)
{
    __shared__ float red[256];
    const int64_t b0 = (int64_t)blockIdx.x * seg;
    const int64_t b1 = b0 + seg < nparts ? b0 + seg : nparts;
    KahanSum acc;
    for (int64_t k = b0 + threadIdx.x; k < b1; k += blockDim.x)
        acc.add(part[k]);
    red[threadIdx.x] = acc.value();
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        out[blockIdx.x] = red[0];
}

// The step count of an Adam state lives on the device with its moments: a
// step is counted, and its bias corrections 1 - beta^t computed, only when
// the batch loss is finite, so that an update skipped for a non-finite loss
// leaves the count where the moments are.  One thread.
__global__ void adam_count_kernel(AdamClock clk, double beta1, double beta2,
                                  const float *__restrict__ loss)
{
    if (!isfinite(loss[0]))
        return;
    const int64_t t = clk.t[0] + 1;
    clk.t[0] = t;
    clk.corr[0] = 1.0 - pow(beta1, (double)t);
    clk.corr[1] = 1.0 - pow(beta2, (double)t);
}

__global__ void adam_kernel(float *__restrict__ params, const float *__restrict__ grad,
                            double *__restrict__ m, double *__restrict__ v, int n, double lr,
                            double beta1, double beta2, double eps,
                            const double *__restrict__ corr, const float *__restrict__ loss)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n || !isfinite(loss[0]))
        return;
    const double c1 = corr[0], c2 = corr[1];
    const double gk = (double)grad[k];
    const double mk = beta1 * m[k] + (1.0 - beta1) * gk;
    const double vk = beta2 * v[k] + (1.0 - beta2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    const double mh = mk / c1, vh = vk / c2;
    params[k] = (float)((double)params[k] - lr * mh / (sqrt(vh) + eps));
}

// ---------------------------------------------------------------------------
// Host helpers
// ---------------------------------------------------------------------------
template <typename Tp> hipError_t grow(Tp **p, size_t count)
{
    (void)hipFree(*p);
    *p = nullptr;
    return hipMalloc((void **)p, count * sizeof(Tp));
}

hipError_t ensure_acts(TrainScratch &s, int64_t n)
{
    hipError_t e = hipSuccess;
    if (!s.grad) {
        if ((e = hipMalloc((void **)&s.grad, FABRIC_N_PARAMS * sizeof(float))) != hipSuccess) return e;
        if ((e = hipMalloc((void **)&s.dcf, FABRIC_MAX_FABRICS * 64 * sizeof(float))) != hipSuccess) return e;
        if ((e = hipMalloc((void **)&s.dz, FABRIC_MAX_FABRICS * kLatent * sizeof(float))) != hipSuccess) return e;
        if ((e = hipMalloc((void **)&s.enc_acts, (size_t)FABRIC_MAX_FABRICS * kEncActFloats * sizeof(float))) != hipSuccess) return e;
        if ((e = hipMalloc((void **)&s.latents, FABRIC_MAX_FABRICS * kLatent * sizeof(float))) != hipSuccess) return e;
        if ((e = hipMalloc((void **)&s.cfold, FABRIC_MAX_FABRICS * 64 * sizeof(float))) != hipSuccess) return e;
        if ((e = hipMalloc((void **)&s.loss, sizeof(float))) != hipSuccess) return e;
        // The largest images are the FP32 ones.
        if ((e = hipMalloc(&s.fwd_image, decoder_image_bytes(FABRIC_FP32))) != hipSuccess) return e;
        if ((e = hipMalloc(&s.bwd_image, (size_t)BwdShape<1>::NFRAG * 64 * sizeof(float))) != hipSuccess) return e;
    }
    // A multiple of 64 samples: whole 32-sample groups of the BF16 planes
    // are read in bounds.
    const int64_t cap = (n + 63) / 64 * 64;
    if (s.cap < cap) {
        if ((e = grow(&s.acts, (size_t)cap * kActFloats)) != hipSuccess) return e;
        // the per-tile parts, then the first stage's sums
        if ((e = grow(&s.loss_part, (size_t)cap / 16 + 1 + kLossStage)) != hipSuccess) return e;
        s.cap = cap;
    }
    return e;
}

hipError_t ensure_partials(TrainScratch &s, int n_jobs, int nblk = kWgBlocks)
{
    const size_t need = (size_t)n_jobs * nblk * kWgMaxM * kWgMaxC;
    if (s.partial_floats >= need)
        return hipSuccess;
    hipError_t e = grow(&s.partials, need);
    if (e == hipSuccess)
        s.partial_floats = need;
    return e;
}

hipError_t pack_images(TrainScratch &s, int prec, const float *dec_params, hipStream_t stream)
{
    hipError_t e = launch_pack_decoder(prec, dec_params, s.fwd_image, stream);
    if (e != hipSuccess)
        return e;
    if (prec == FABRIC_FP32) {
        const int total = BwdShape<1>::NFRAG * 64;
        hipLaunchKernelGGL(pack_backward_kernel<FABRIC_FP32>, dim3((total + 255) / 256), dim3(256), 0,
                           stream, dec_params, (float *)s.bwd_image);
    } else {
        const int total = BwdShape<8>::NFRAG * 64;
        hipLaunchKernelGGL(pack_backward_kernel<FABRIC_BF16>, dim3((total + 255) / 256), dim3(256), 0,
                           stream, dec_params, (bf16x8 *)s.bwd_image);
    }
    return hipGetLastError();
}

template <int P, bool GIVEN>
hipError_t launch_fwd_bwd(TrainScratch &s, const fabric_gbuffer &g, const DevFabric *fabrics,
                          int n_fabrics, const float *cfold, const float *tgt_or_dy,
                          unsigned long long *err, hipStream_t stream)
{
    using M = Mfma<P>;
    using S = DecShape<M::KPL>;
    const auto *ffr = (const typename M::Frag *)s.fwd_image;
    const auto *fb = (const f32x4 *)((const char *)s.fwd_image + (size_t)S::NFRAG * 64 * sizeof(typename M::Frag));
    const auto *bfr = (const typename M::Frag *)s.bwd_image;
    const int64_t tiles = (g.n + 15) / 16;
    const int64_t blocks = (tiles + 3) / 4;
    hipLaunchKernelGGL((fwd_bwd_kernel<P, GIVEN>), dim3((unsigned)blocks), dim3(256), 0, stream, g,
                       fabrics, n_fabrics, cfold, ffr, fb, bfr, tgt_or_dy, s.acts, s.cap,
                       s.loss_part, err);
    return hipGetLastError();
}

// Weight gradients of the decoder from the per-sample rows: writes every
// decoder tensor of grad_dec except W1's latent columns, plus dcf.
// The same from the BF16 planes of a BF16 training step.
hipError_t decoder_weight_grads_bf16(TrainScratch &s, const fabric_gbuffer &g, int n_fabrics,
                                     float *grad_dec, hipStream_t stream)
{
    const int64_t n = g.n;
    WgJobs16 jobs{};
    WgDests dests{};
    int nj = 0;
    auto add = [&](int A, int MA, int B, int NB, int bias, const uint16_t *ids,
                   int f0, int NC, float *dst, int ldw, float *bsum, int transposed) {
        jobs.j[nj] = WgJob16{A, B, ids, MA, NB, bias, f0, NC};
        dests.d[nj] = WgDest{dst, bsum, MA, NC, ids ? NC : NB, ldw, transposed};
        nj++;
    };
    add(kQDH1, 64, kQS, 40, 1, nullptr, 0, 41, grad_dec + kOffW1 + kLatent, 72,
        grad_dec + kOffB1, 0);
    add(kQDH2, 64, kQH1, 64, 1, nullptr, 0, 65, grad_dec + kOffW2, 64, grad_dec + kOffB2, 0);
    add(kQDH3, 64, kQX3, 69, 1, nullptr, 0, 70, grad_dec + kOffW3, 69, grad_dec + kOffB3, 0);
    add(kQDY, 4, kQH3, 64, 1, nullptr, 0, 65, grad_dec + kOffW4, 64, grad_dec + kOffB4, 0);
    for (int f0 = 0; f0 < n_fabrics; f0 += 64) {
        const int NC = n_fabrics - f0 < 64 ? n_fabrics - f0 : 64;
        add(kQDH1, 64, -1, 0, 0, g.fabric_id, f0, NC, s.dcf + f0 * 64, 64, nullptr, 1);
    }
    hipError_t e = ensure_partials(s, nj);
    if (e != hipSuccess)
        return e;
    int64_t per_block = (n + kWgBlocks - 1) / kWgBlocks;
    per_block = (per_block + 63) / 64 * 64;
    hipLaunchKernelGGL(wgrad_bf16_kernel, dim3(kWgBlocks, nj), dim3(256), 0, stream, jobs, n,
                       (const __bf16 *)s.acts, per_block, s.partials);
    hipLaunchKernelGGL(wgrad_reduce_kernel,
                       dim3((kWgMaxM * kWgMaxC + kWgRedEntries - 1) / kWgRedEntries, nj), dim3(256), 0,
                       stream, (const float *)s.partials, dests, kWgBlocks);
    return hipGetLastError();
}

// Output tiles of the fused launch's weight gradients: W1 (4 x 3), W2 and W3
// (4 x 5 each), W4 (1 x 5), and 4 per 16 fabrics of dL/dc_f.
int fused_tile_count(int n_fabrics)
{
    int tiles = 4 * 3 + 4 * 5 + 4 * 5 + 1 * 5;
    for (int f0 = 0; f0 < n_fabrics; f0 += 64) {
        const int NC = n_fabrics - f0 < 64 ? n_fabrics - f0 : 64;
        tiles += 4 * ((NC + 15) / 16);
    }
    return tiles;
}
bool fused_fits(int n_fabrics) { return fused_tile_count(n_fabrics) <= kFMaxSlots * kFWaves; }

// BF16 training's forward, loss, backward and decoder weight gradients in
// one persistent launch (train_bf16_fused_kernel), then the partials' sums:
// writes the loss parts, every decoder tensor of grad_dec except W1's latent
// columns, and dcf.
hipError_t train_bf16_fused(TrainScratch &s, const fabric_gbuffer &g, const DevFabric *fabrics,
                            int n_fabrics, const float *targets, unsigned long long *err,
                            float *grad_dec, int64_t *loss_parts, hipStream_t stream)
{
    FusedJobs jobs{};
    WgDests dests{};
    int nj = 0, tiles = 0;
    auto add = [&](int A, int MA, int B, int NB, int bias, int f0, int NC, float *dst, int ldw,
                   float *bsum, int transposed) {
        jobs.j[nj] = WgJob16{A, B, B < 0 ? g.fabric_id : nullptr, MA, NB, bias, f0, NC};
        dests.d[nj] = WgDest{dst, bsum, MA, NC, B < 0 ? NC : NB, ldw, transposed};
        jobs.first_tile[nj] = tiles;
        tiles += ((MA + 15) / 16) * ((NC + 15) / 16);
        nj++;
    };
    add(kQDH1, 64, kQS, 40, 1, 0, 41, grad_dec + kOffW1 + kLatent, 72, grad_dec + kOffB1, 0);
    add(kQDH2, 64, kQH1, 64, 1, 0, 65, grad_dec + kOffW2, 64, grad_dec + kOffB2, 0);
    add(kQDH3, 64, kQX3, 69, 1, 0, 70, grad_dec + kOffW3, 69, grad_dec + kOffB3, 0);
    add(kQDY, 4, kQH3, 64, 1, 0, 65, grad_dec + kOffW4, 64, grad_dec + kOffB4, 0);
    for (int f0 = 0; f0 < n_fabrics; f0 += 64) {
        const int NC = n_fabrics - f0 < 64 ? n_fabrics - f0 : 64;
        add(kQDH1, 64, -1, 0, 0, f0, NC, s.dcf + f0 * 64, 64, nullptr, 1);
    }
    jobs.first_tile[nj] = tiles;
    jobs.n_jobs = nj;
    if (tiles != fused_tile_count(n_fabrics) || tiles > kFMaxSlots * kFWaves)
        return hipErrorInvalidValue;
    hipError_t e;
    if (s.n_cu == 0) {
        int dev = 0;
        if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
        if ((e = hipDeviceGetAttribute(&s.n_cu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
            return e;
        if ((e = hipFuncSetAttribute((const void *)train_bf16_fused_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFLds)) != hipSuccess)
            return e;
    }
    const int64_t n_chunks = (g.n + kFChunk - 1) / kFChunk;
    const int grid = (int)(n_chunks < s.n_cu ? n_chunks : s.n_cu);   // one block per CU
    if ((e = ensure_partials(s, nj, grid)) != hipSuccess)
        return e;
    *loss_parts = grid;          // one loss part per block
    using M = Mfma<FABRIC_BF16>;
    using S = DecShape<M::KPL>;
    const auto *ffr = (const bf16x8 *)s.fwd_image;
    const auto *fb = (const f32x4 *)((const char *)s.fwd_image + (size_t)S::NFRAG * 64 * sizeof(bf16x8));
    hipLaunchKernelGGL(train_bf16_fused_kernel, dim3(grid), dim3(64 * kFWaves), kFLds, stream, g,
                       fabrics, n_fabrics, (const float *)s.cfold, ffr, fb,
                       (const bf16x8 *)s.bwd_image, targets, s.loss_part, err, jobs, n_chunks,
                       s.partials);
    hipLaunchKernelGGL(wgrad_reduce_kernel,
                       dim3((kWgMaxM * kWgMaxC + kWgRedEntries - 1) / kWgRedEntries, nj), dim3(256), 0,
                       stream, (const float *)s.partials, dests, grid);
    return hipGetLastError();
}

hipError_t decoder_weight_grads(TrainScratch &s, const fabric_gbuffer &g, int n_fabrics,
                                float *grad_dec, hipStream_t stream)
{
    const int64_t n = g.n;
    ActPtrs ap = act_ptrs(s.acts, s.cap);
    WgJobs jobs{};
    WgDests dests{};
    int nj = 0;
    auto add = [&](const float *A, int lda, int MA, const float *B, int ldb, int NB, int bias,
                   const uint16_t *ids, int f0, int NC, float *dst, int ldw, float *bsum,
                   int transposed) {
        jobs.j[nj] = WgJob{A, B, ids, lda, MA, ldb, NB, bias, f0, NC};
        dests.d[nj] = WgDest{dst, bsum, MA, NC, ids ? NC : NB, ldw, transposed};
        nj++;
    };
    add(ap.DH1, kDH, 64, ap.S, kS, 40, 1, nullptr, 0, 41, grad_dec + kOffW1 + kLatent, 72,
        grad_dec + kOffB1, 0);
    add(ap.DH2, kDH, 64, ap.H1, kH1, 64, 1, nullptr, 0, 65, grad_dec + kOffW2, 64, grad_dec + kOffB2, 0);
    add(ap.DH3, kDH, 64, ap.X3, kX3, 69, 1, nullptr, 0, 70, grad_dec + kOffW3, 69, grad_dec + kOffB3, 0);
    add(ap.DY, kDY, 4, ap.H3, kH3, 64, 1, nullptr, 0, 65, grad_dec + kOffW4, 64, grad_dec + kOffB4, 0);
    // dL/dc_f: segment sums of dh1 by fabric (one-hot B), up to 64 fabrics per job.
    for (int f0 = 0; f0 < n_fabrics; f0 += 64) {
        const int NC = n_fabrics - f0 < 64 ? n_fabrics - f0 : 64;
        add(ap.DH1, kDH, 64, nullptr, 0, 0, 0, g.fabric_id, f0, NC, s.dcf + f0 * 64, 64, nullptr, 1);
    }
    hipError_t e = ensure_partials(s, nj);
    if (e != hipSuccess)
        return e;
    int64_t per_block = (n + kWgBlocks - 1) / kWgBlocks;
    per_block = (per_block + 63) / 64 * 64;
    hipLaunchKernelGGL(wgrad_kernel, dim3(kWgBlocks, nj), dim3(256), 0, stream, jobs, n, per_block,
                       s.partials);
    hipLaunchKernelGGL(wgrad_reduce_kernel,
                       dim3((kWgMaxM * kWgMaxC + kWgRedEntries - 1) / kWgRedEntries, nj), dim3(256), 0,
                       stream, (const float *)s.partials, dests, kWgBlocks);
    return hipGetLastError();
}

hipError_t run_encoder_backward(TrainScratch &s, const float *enc_params, const float *enc_inputs,
                                int n_fabrics, const float *dz, float *grad_enc, hipStream_t stream)
{
    hipLaunchKernelGGL(encoder_backward_kernel, dim3(n_fabrics), dim3(kEncThreads), 0, stream, enc_params,
                       enc_inputs, dz, s.enc_acts);
    hipLaunchKernelGGL(encoder_wgrad_kernel, dim3((kNEnc + 255) / 256), dim3(256), 0, stream,
                       (const float *)s.enc_acts, n_fabrics, grad_enc);
    return hipGetLastError();
}

}  // namespace

void train_scratch_free(TrainScratch &s)
{
    (void)hipFree(s.acts);
    (void)hipFree(s.loss_part);
    (void)hipFree(s.partials);
    (void)hipFree(s.grad);
    (void)hipFree(s.dcf);
    (void)hipFree(s.dz);
    (void)hipFree(s.enc_acts);
    (void)hipFree(s.latents);
    (void)hipFree(s.cfold);
    (void)hipFree(s.fwd_image);
    (void)hipFree(s.bwd_image);
    (void)hipFree(s.loss);
    (void)hipFree(s.b_fid);
    (void)hipFree(s.b_fields);
    (void)hipFree(s.targets);
    s = TrainScratch();
}

hipError_t launch_adam(float *params, const float *grad, double *m, double *v, int n,
                       const fabric_train_cfg &cfg, AdamClock clk, const float *loss,
                       hipStream_t stream)
{
    hipLaunchKernelGGL(adam_count_kernel, dim3(1), dim3(1), 0, stream, clk, cfg.beta1, cfg.beta2,
                       loss);
    hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, params, grad, m, v,
                       n, cfg.lr, cfg.beta1, cfg.beta2, cfg.eps, (const double *)clk.corr, loss);
    return hipGetLastError();
}

hipError_t launch_make_batch(uint64_t seed, int64_t n, int n_fabrics, float r_lo, float r_hi,
                             float btdf_frac, const fabric_gbuffer_out &out, hipStream_t stream)
{
    if (n <= 0)
        return hipSuccess;
    const double lo = std::log((double)r_lo), hi = std::log((double)r_hi);
    hipLaunchKernelGGL(make_batch_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                       seed, n, n_fabrics, (float)lo, (float)(hi - lo), btdf_frac, out);
    return hipGetLastError();
}

hipError_t decoder_backward(TrainScratch &s, const fabric_gbuffer &g, const DevFabric *fabrics,
                            int n_fabrics, const float *dec_params, const float *latents,
                            const float *grad_y4, float *grad_params, float *grad_latents,
                            hipStream_t stream)
{
    hipError_t e = ensure_acts(s, g.n > 0 ? g.n : 1);
    if (e != hipSuccess) return e;
    if ((e = pack_images(s, FABRIC_FP32, dec_params, stream)) != hipSuccess) return e;
    if ((e = launch_fold_latents(dec_params, latents, n_fabrics, s.cfold, stream)) != hipSuccess) return e;
    if (g.n > 0) {
        if ((e = launch_fwd_bwd<FABRIC_FP32, true>(s, g, fabrics, n_fabrics, s.cfold, grad_y4, nullptr,
                                                   stream)) != hipSuccess)
            return e;
        if ((e = decoder_weight_grads(s, g, n_fabrics, grad_params, stream)) != hipSuccess) return e;
    } else {
        if ((e = hipMemsetAsync(grad_params, 0, FABRIC_N_DECODER_PARAMS * sizeof(float), stream)) != hipSuccess) return e;
        if ((e = hipMemsetAsync(s.dcf, 0, (size_t)n_fabrics * 64 * sizeof(float), stream)) != hipSuccess) return e;
    }
    const int tot = (n_fabrics * kLatent > 64 * kLatent) ? n_fabrics * kLatent : 64 * kLatent;
    hipLaunchKernelGGL(latent_grads_kernel, dim3((tot + 255) / 256), dim3(256), 0, stream, dec_params,
                       (const float *)s.dcf, latents, n_fabrics, grad_latents, grad_params + kOffW1);
    return hipGetLastError();
}

hipError_t encoder_backward(TrainScratch &s, const float *enc_params, const float *enc_inputs,
                            int n_fabrics, const float *grad_latents, float *grad_enc_params,
                            hipStream_t stream)
{
    hipError_t e = ensure_acts(s, 1);
    if (e != hipSuccess)
        return e;
    return run_encoder_backward(s, enc_params, enc_inputs, n_fabrics, grad_latents,
                                grad_enc_params, stream);
}

namespace {

// Loss and full gradient (into s.grad) of one batch; s.loss holds the loss.
hipError_t loss_and_grad(TrainScratch &s, const TrainArgs &a, hipStream_t stream)
{
    const fabric_train_cfg &cfg = a.cfg;
    fabric_gbuffer g;
    hipError_t e;
    if (a.batch) {
        g = *a.batch;
    } else {
        const int64_t n = cfg.batch;
        if (s.batch_cap < n) {
            if ((e = grow(&s.b_fid, (size_t)n)) != hipSuccess) return e;
            if ((e = grow(&s.b_fields, (size_t)n * 9)) != hipSuccess) return e;
            if ((e = grow(&s.targets, (size_t)n * 4)) != hipSuccess) return e;
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
    if ((e = ensure_acts(s, n > 0 ? n : 1)) != hipSuccess) return e;
    const float *targets = a.targets;
    if (!targets && n > 0) {
        if (s.batch_cap < n) {
            // A caller-supplied batch larger than any generated one: the
            // batch planes are not in use, so all three buffers may grow.
            if ((e = grow(&s.targets, (size_t)n * 4)) != hipSuccess) return e;
            if ((e = grow(&s.b_fid, (size_t)n)) != hipSuccess) return e;
            if ((e = grow(&s.b_fields, (size_t)n * 9)) != hipSuccess) return e;
            s.batch_cap = n;
        }
        if ((e = launch_gt_filter(g, a.fabrics, a.n_fabrics, cfg.gt_samples, cfg.seed ^ 1ull, a.vis,
                                  nullptr, s.targets, a.err, stream)) != hipSuccess)
            return e;
        targets = s.targets;
    }
    const float *dec = a.params, *enc = a.params + kNDec;
    if ((e = launch_encoder_forward(enc, a.enc_inputs, a.n_fabrics, s.latents, stream)) != hipSuccess) return e;
    if ((e = launch_fold_latents(dec, s.latents, a.n_fabrics, s.cfold, stream)) != hipSuccess) return e;
    if ((e = pack_images(s, cfg.prec, dec, stream)) != hipSuccess) return e;
    if (n > 0) {
        // Faults of a generated-target batch were counted by the filter.
        unsigned long long *err = a.targets ? a.err : nullptr;
        // BF16 with at most 16 fabrics: one fused launch, the activations kept
        // on chip; otherwise the blocked BF16 planes through HBM.
        const bool fused = cfg.prec == FABRIC_BF16 && fused_fits(a.n_fabrics);
        int64_t parts = (n + 15) / 16;       // one loss part per 16-sample tile
        e = cfg.prec == FABRIC_FP32
                ? launch_fwd_bwd<FABRIC_FP32, false>(s, g, a.fabrics, a.n_fabrics, s.cfold, targets, err, stream)
            : fused ? train_bf16_fused(s, g, a.fabrics, a.n_fabrics, targets, err, s.grad, &parts, stream)
                    : launch_fwd_bwd<FABRIC_BF16, false>(s, g, a.fabrics, a.n_fabrics, s.cfold, targets, err, stream);
        if (e != hipSuccess) return e;
        if (parts <= 4096) {
            hipLaunchKernelGGL(loss_reduce_kernel, dim3(1), dim3(256), 0, stream,
                               (const float *)s.loss_part, parts, 1.0f / (float)n, s.loss);
        } else {
            // Large batches: fixed segments summed by up to kLossStage blocks first.
            const int64_t seg = (parts + kLossStage - 1) / kLossStage;
            const int64_t nb = (parts + seg - 1) / seg;
            float *stage = s.loss_part + s.cap / 16 + 1;
            hipLaunchKernelGGL(loss_stage_kernel, dim3((unsigned)nb), dim3(256), 0, stream,
                               (const float *)s.loss_part, parts, seg, stage);
            hipLaunchKernelGGL(loss_reduce_kernel, dim3(1), dim3(256), 0, stream,
                               (const float *)stage, nb, 1.0f / (float)n, s.loss);
        }
        if (!fused) {
            e = cfg.prec == FABRIC_FP32 ? decoder_weight_grads(s, g, a.n_fabrics, s.grad, stream)
                                        : decoder_weight_grads_bf16(s, g, a.n_fabrics, s.grad, stream);
            if (e != hipSuccess) return e;
        }
    } else {
        if ((e = hipMemsetAsync(s.loss, 0, sizeof(float), stream)) != hipSuccess) return e;
        if ((e = hipMemsetAsync(s.grad, 0, kNDec * sizeof(float), stream)) != hipSuccess) return e;
        if ((e = hipMemsetAsync(s.dcf, 0, (size_t)a.n_fabrics * 64 * sizeof(float), stream)) != hipSuccess) return e;
    }
    const int tot = (a.n_fabrics * kLatent > 64 * kLatent) ? a.n_fabrics * kLatent : 64 * kLatent;
    hipLaunchKernelGGL(latent_grads_kernel, dim3((tot + 255) / 256), dim3(256), 0, stream, dec,
                       (const float *)s.dcf, (const float *)s.latents, a.n_fabrics, s.dz, s.grad + kOffW1);
    if ((e = run_encoder_backward(s, enc, a.enc_inputs, a.n_fabrics, s.dz, s.grad + kNDec, stream)) != hipSuccess)
        return e;
    return hipGetLastError();
}

hipError_t read_loss(TrainScratch &s, float *out_loss, int *finite_loss, hipStream_t stream)
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

hipError_t loss_grad(TrainScratch &s, const TrainArgs &a, float *grad_out, float *out_loss,
                     hipStream_t stream)
{
    hipError_t e = loss_and_grad(s, a, stream);
    if (e != hipSuccess)
        return e;
    if ((e = hipMemcpyAsync(grad_out, s.grad, FABRIC_N_PARAMS * sizeof(float), hipMemcpyDeviceToDevice,
                            stream)) != hipSuccess)
        return e;
    if (out_loss) {
        int fin = 0;
        return read_loss(s, out_loss, &fin, stream);
    }
    return hipSuccess;
}

hipError_t train_step(TrainScratch &s, const TrainArgs &a, float *out_loss, int *updated,
                      hipStream_t stream)
{
    *updated = 1;
    const fabric_train_cfg &cfg = a.cfg;
    hipError_t e = loss_and_grad(s, a, stream);
    if (e != hipSuccess)
        return e;
    if ((e = launch_adam(a.params, (const float *)s.grad, a.adam_m, a.adam_v, FABRIC_N_PARAMS, cfg,
                         a.clock, (const float *)s.loss, stream)) != hipSuccess)
        return e;
    if (out_loss)
        return read_loss(s, out_loss, updated, stream);
    return hipSuccess;
}

}  // namespace fab
