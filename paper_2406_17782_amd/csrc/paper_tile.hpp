// The paper-size decoder on 32x32x16 MFMA tiles (BF16 / FP16 operands, FP32
// accumulation), shared by its shading and its training kernels: the
// fragment image's layout, the one-blob slots of a lane group and the
// operand packing.  32-pixel tiles in the layout of the config decoder's
// shading kernel (lane group g = l/32 owns chained neurons
// 32 mb + 8 (r/4) + 4 g + r%4; one layer's output is the next layer's B
// operand without data movement); each layer's bias rides in a K slot that
// holds 1 (the first extra slot of lane group 0): F1's bias is folded with
// the latent into the per-fabric C operand c_f, A1's extra slots carry
// wi.xyz / wo.xy / 1 as in the config decoder, A3's C operand is the
// residual input, A5's bias is added after the MFMA.
#pragma once

#include "mlp_tile32.hpp"
#include "paper_net.hpp"

namespace fab {

// Fragment image: [layer][M-block][k-step] A fragments of 64 lanes x 8 bf16.
// K steps: F1 2 (12 slots: 8 position bins, 4 size bins), chain layers 5
// (32 chained neurons + the bias slot), A1 5 (32 + wi.xyz | wo.xy, 1), A5 4.
enum PLayer { kF1 = 0, kF2, kA1, kA2, kA3, kA4, kA5, kPLayers };
__host__ __device__ constexpr int p_ks(int l) { return l == kF1 ? 2 : (l == kA5 ? 4 : 5); }
__host__ __device__ constexpr int p_mb(int l) { return l == kA5 ? 1 : 2; }
__host__ __device__ constexpr int p_first(int l)
{
    return l == 0 ? 0 : p_first(l - 1) + p_mb(l - 1) * p_ks(l - 1);
}
constexpr int kPFrags = p_first(kPLayers);     // 58
static_assert(kPFrags == 58, "fragment count");
constexpr int kPSlots1 = 12;                   // F1 slots per lane group

// F1 slot c of lane group g: position bin c of axis g (c < 8), size bin
// 4 g + c - 8 (c < 12); blob channel index [u 0..7, v 8..15, size 16..23].
__host__ __device__ inline int p_blob_channel(int g, int c)
{
    if (c < 8)
        return 8 * g + c;
    if (c < kPSlots1)
        return 16 + 4 * g + (c - 8);
    return -1;
}

// Without the spatial fusion stage (the ablation of Sec. 5 "Spatial
// fusion"), F1 slots 12 .. 14 of lane group 0 carry wi.xyz and slots 12 .. 13
// of group 1 wo.xy, weighted by A1's angular columns; returns the angular
// input 0 .. 4 of F1 slot c, or -1.
__host__ __device__ inline int p_f1_angular(int g, int c)
{
    if (c < kPSlots1 || c >= kPSlots1 + (g == 0 ? 3 : 2))
        return -1;
    return 3 * g + (c - kPSlots1);
}

// One-blob slots of lane group g: 8 circular position bins along its axis,
// then 4 of the 8 size bins (exp(-d^2/2), d in bins).  RAW (the footprint
// encoding's ablation): the position fraction of the group's axis in its
// first bin's slot and, in group 0, tau in the first size bin's slot.
template <int P, bool RAW, int NS>
__device__ inline void paper_slots(float coord, float iper, float r, int g, float (&s1)[NS])
{
    using FM = FeatureMath<P>;
#pragma unroll
    for (int c = kPSlots1; c < NS; c++)
        s1[c] = 0.0f;
    if (RAW) {
#pragma unroll
        for (int c = 0; c < kPSlots1; c++)
            s1[c] = 0.0f;
        s1[0] = coord * iper;
        if (g == 0)
            s1[8] = fminf(fmaxf((FM::log2(r) + 14.0f) * (1.0f / 16.0f), 0.0f), 1.0f);
        return;
    }
    const float t0 = 8.0f * (coord * iper) - 0.5f;
#pragma unroll
    for (int b = 0; b < 8; b++) {
        float d = t0 - (float)b;                       // in [-7.5, 7.5)
        d -= 8.0f * floorf((d + 4.0f) * 0.125f);       // circular, in [-4, 4)
        s1[b] = FM::gauss(d);
    }
    const float tau = fminf(fmaxf((FM::log2(r) + 14.0f) * (1.0f / 16.0f), 0.0f), 1.0f);
#pragma unroll
    for (int b = 0; b < 4; b++)
        s1[8 + b] = FM::gauss(8.0f * tau - (float)(4 * g + b) - 0.5f);
}

// The leaky ReLU with slope k splits as lrelu(x) = s (|x| + c x) with
// s = (1 - k)/2 and c = (1 + k)/(1 - k).  The tile computes the scaled
// activation |x| + c x = lrelu(x)/s in FP32 as one FMA with an
// absolute-value source (a multiply and a max would take three
// instructions: the max also quiets a signalling NaN of the MFMA result),
// and the packed image carries the factor s in the weights that read it
// (see paper_weight_scale).
constexpr float kActS = 0.5f * (1.0f - kLeak);
constexpr float kActC = (1.0f + kLeak) / (1.0f - kLeak);
__device__ inline float lrelu_scaled(float x) { return fmaf(x, kActC, fabsf(x)); }

// Factors of the packed image for layer l's chained weight columns and for
// its bias, so that every layer sees its inputs as the FP32 network does.
// The residual block's input x is scaled (x/s) in both images: it is A2's B
// operand (A2's weights times s) and A3's C operand, so A3's output and
// bias are kept at scale 1/s.  BF16 scales every activation: F2, A1's
// spatial columns and A5 read one scaled activation (s); A3 reads the
// scaled A2 activation (1); A4 reads an activation scaled by 1/s^2 (s^2).
// FP16 activates on packed halves without scaling: A3 reads a plain one
// (1/s) and A4 one scaled by 1/s through A3's output (s).  F1, the angular
// columns and A5's bias (added after the MFMA) are unscaled.
__host__ __device__ inline float paper_weight_scale(int P, int l)
{
    if (P == FABRIC_BF16)
        return l == kF1 || l == kA3 ? 1.0f : l == kA4 ? kActS * kActS : kActS;
    return l == kA2 || l == kA4 ? kActS : l == kA3 ? 1.0f / kActS : 1.0f;
}
__host__ __device__ inline float paper_bias_scale(int, int l)
{
    return l == kA3 ? 1.0f / kActS : 1.0f;
}

// Operand packing and the MFMA sweep per operand precision.  act(): the
// leaky ReLU fused into the packing of eight outputs - in FP32 before the
// BF16 rounding as the scaled activation above (CDNA has no packed BF16
// arithmetic), on packed halves after the FP16 rounding (packed multiply and
// max, two values per instruction).
template <int P> struct PaperTile {
    using M = Mfma<P>;
    using Frag = typename M::Frag;

    // The residual block's input, in place: the scaled activation, in FP32.
    static __device__ inline void act_acc(f32x16 (&a)[2])
    {
#pragma unroll
        for (int mb = 0; mb < 2; mb++)
#pragma unroll
            for (int r = 0; r < 16; r++)
                a[mb][r] = lrelu_scaled(a[mb][r]);
    }

    template <int NSL> static __device__ inline Frag frag_of(const float (&v)[NSL], int ks, bool act)
    {
        f32x8 x;
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const int c = ks * 8 + j;
            x[j] = c < NSL ? v[c] : 0.0f;
        }
        if (P == FABRIC_FP16) {
            Frag f = M::from8(x);
            if (act)
                f = __builtin_elementwise_max(f, f * (Frag)((_Float16)kLeak));
            return f;
        }
        if (act) {
#pragma unroll
            for (int j = 0; j < 8; j++)
                x[j] = P == FABRIC_BF16 ? lrelu_scaled(x[j]) : lrelu(x[j]);
        }
        return M::from8(x);
    }

    // The chained B operand of a 64-neuron layer output.
    static __device__ inline void chain_b(const f32x16 (&a)[2], Frag (&B)[4], bool act)
    {
        float v[kChain32];
#pragma unroll
        for (int c = 0; c < kChain32; c++)
            v[c] = a[c >> 4][c & 15];
#pragma unroll
        for (int ks = 0; ks < 4; ks++)
            B[ks] = frag_of(v, ks, act);
    }

    // acc[t][mb] += A(layer, mb, ks) B[t][ks] over the layer's K steps for
    // the T tiles in flight: each A fragment is read from LDS once and used
    // by all T.
    template <int T, int NMB, int KS>
    static __device__ inline void dense_lds(const Frag *__restrict__ s_w, int first,
                                            const Frag (&B)[T][KS], f32x16 (&acc)[T][2], int lane)
    {
#pragma unroll
        for (int ks = 0; ks < KS; ks++)
#pragma unroll
            for (int mb = 0; mb < NMB; mb++) {
                const Frag w = s_w[(first + mb * KS + ks) * 64 + lane];
#pragma unroll
                for (int t = 0; t < T; t++)
                    acc[t][mb] = Mfma32<P>::mma(w, B[t][ks], acc[t][mb]);
            }
    }
};

}  // namespace fab
