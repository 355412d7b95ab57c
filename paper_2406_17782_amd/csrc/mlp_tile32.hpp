// Decoder tile of 32 pixels on 32x32x16 MFMA (bf16 / fp16 operands), the
// shading kernel's layout.  Compared with 16-pixel tiles, two lane groups
// instead of four share a pixel, so the per-pixel work (loads, checks, input
// encoding set-up, output decoding) is replicated half as often, and the
// first and third layers pad K less (48 and 40 instead of 64 and 96).
//
// Per the CDNA 32x32x16 layout (checked on the device), lane l holds
// A[m = l%32][k = 8*(l/32) + j], B[k = 8*(l/32) + j][n = l%32] and
// D[m = 8*(r/4) + 4*(l/32) + r%4][n = l%32] in accumulator register r.
// Lane group g = l/32 therefore owns neurons 32*mb + 8*(r/4) + 4*g + r%4 of
// each 32-row M-block mb, and slot c (k-step c/8, position c%8) of the next
// layer carries neuron 32*(c/16) + 8*((c%16)/4) + 4*g + c%4: the output of
// one layer is the next layer's B operand without data movement.
//
// Slots per lane group g:
//   L1: c = 0..7 sin 2 pi frac(2^c p_g), c = 8..15 the cosines, c = 16..19
//       one-blob bins 4g..4g+3, c = 20..23 zero (p_0 = u, p_1 = v tiled)
//   L2, L4: c = 0..31 chained neurons
//   L3: c = 0..31 chained neurons; c = 32..34: g = 0 (wi.x, wi.y, wi.z),
//       g = 1 (wo.x, wo.y, 1), the constant 1 carrying the layer's bias
#pragma once

#include "mlp_tile.hpp"

namespace fab {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kL1Slots32 = 20;
constexpr int kChain32 = 32;
constexpr int kL3Slots32 = 35;

__host__ __device__ inline int chain32_neuron(int g, int c)
{
    return 32 * (c >> 4) + 8 * ((c & 15) >> 2) + 4 * g + (c & 3);
}

// Spatial-feature index (0..39) of L1 slot c of lane group g, or -1.
__host__ __device__ inline int l1_feature32(int g, int c)
{
    if (c < 8)
        return 16 * g + c;
    if (c < 16)
        return 16 * g + 8 + (c - 8);
    if (c < kL1Slots32)
        return 32 + 4 * g + (c - 16);
    return -1;
}

// L3 slot 32 + a of lane group g: angular input 0..4 (wi.x, wi.y, wi.z, wo.x,
// wo.y), 5 for the bias slot, -1 for zero.
__host__ __device__ inline int l3_extra32(int g, int a)
{
    if (a > 2)
        return -1;
    return g == 0 ? a : (a < 2 ? 3 + a : 5);
}

template <int KPL> struct DecShape32 {
    static_assert(KPL == 8, "32x32x16 operands");
    static constexpr int KS1 = div_up(kL1Slots32, 8);    // 3
    static constexpr int KS2 = div_up(kChain32, 8);      // 4
    static constexpr int KS3 = div_up(kL3Slots32, 8);    // 5
    static constexpr int KS4 = div_up(kChain32, 8);      // 4
    static constexpr int FRAG_L1 = 0;                    // 2 M-blocks each
    static constexpr int FRAG_L2 = FRAG_L1 + 2 * KS1;
    static constexpr int FRAG_L3 = FRAG_L2 + 2 * KS2;
    static constexpr int FRAG_L4 = FRAG_L3 + 2 * KS3;    // 1 M-block (rows 0..3)
    static constexpr int NFRAG = FRAG_L4 + KS4;          // 28
};

template <int P> struct Mfma32;
template <> struct Mfma32<FABRIC_BF16> {
    static __device__ inline f32x16 mma(bf16x8 a, bf16x8 b, f32x16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma32<FABRIC_FP16> {
    static __device__ inline f32x16 mma(f16x8 a, f16x8 b, f32x16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};

// Packed decoder image of the 32-pixel layout: A fragments [NFRAG][64][8],
// then the L2 C-operand bias [2 M-blocks][64 lanes][16] and the L4 one
// [64 lanes][4] (rows 0..3 in lane group 0).
template <int P> struct Tile32 {
    using M = Mfma<P>;
    using Frag = typename M::Frag;
    using S = DecShape32<8>;
    using FM = FeatureMath<P>;

    template <int NSL>
    static __device__ inline Frag frag_of(const float (&vals)[NSL], int ks)
    {
        f32x8 v;
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const int c = ks * 8 + j;
            v[j] = c < NSL ? vals[c] : 0.0f;
        }
        return M::from8(v);
    }

    // L1 slot values for lane group g (see the header comment).
    static __device__ inline void spatial_slots(float u, float v, float r, float fwx, float fwy,
                                                float iwx, float iwy, int g,
                                                float (&s1)[kL1Slots32])
    {
        const float per = g ? fwy : fwx;
        const float iper = g ? iwy : iwx;
        const float ph = wrap_period(g ? v : u, per, iper) * iper;
        float sn, cs;
        FM::sincos2pi(ph, &sn, &cs);
#pragma unroll
        for (int q = 0; q < 8; q++) {
            s1[q] = sn;
            s1[8 + q] = cs;
            // angle doubling: sin 2x = 2 sin x cos x, cos 2x = 1 - 2 sin^2 x
            // (three instructions; the negation is a free source modifier)
            const float t = sn + sn;
            cs = fmaf(-t, sn, 1.0f);
            sn = t * s1[8 + q];
        }
        const float tau = fminf(fmaxf((FM::log2(r) + 14.0f) * (1.0f / 16.0f), 0.0f), 1.0f);
#pragma unroll
        for (int b = 0; b < 4; b++)
            s1[16 + b] = FM::gauss(8.0f * tau - (float)(4 * g + b) - 0.5f);
    }

    template <int KS>
    static __device__ inline void chain(const f32x16 (&acc)[2], Frag (&B)[KS])
    {
        float v[kChain32];
#pragma unroll
        for (int c = 0; c < kChain32; c++)
            v[c] = acc[c >> 4][c & 15];
#pragma unroll
        for (int ks = 0; ks < KS; ks++)
            B[ks] = M::relu(frag_of(v, ks));
    }

    template <int NMB, int KS, typename GetA>
    static __device__ inline void dense(GetA getA, int base, const Frag (&B)[KS], f32x16 (&acc)[2])
    {
#pragma unroll
        for (int mb = 0; mb < NMB; mb++)
#pragma unroll
            for (int ks = 0; ks < KS; ks++)
                acc[mb] = Mfma32<P>::mma(getA(base + mb * KS + ks), B[ks], acc[mb]);
    }

    // L3 slots: chained neurons (rectified), then the three extra inputs.
    static __device__ inline void l3_frags(const f32x16 (&a)[2], float x0, float x1, float x2,
                                           Frag (&B3)[S::KS3])
    {
        float v[kL3Slots32];
#pragma unroll
        for (int c = 0; c < kChain32; c++)
            v[c] = a[c >> 4][c & 15];
        v[32] = x0;
        v[33] = x1;
        v[34] = x2;
#pragma unroll
        for (int ks = 0; ks < S::KS3; ks++) {
            B3[ks] = frag_of(v, ks);
            if ((ks + 1) * 8 <= kChain32)
                B3[ks] = M::relu(B3[ks]);
        }
    }

    // Forward: cf / b2 are the L1 / L2 C operands (per lane, both M-blocks).
    // Returns W4 h3 (without its bias) in accumulator registers 0..3 of lane
    // group 0; L4 starts from a zero C operand, which saves the sixteen
    // registers a bias operand would hold for four useful rows.
    template <typename GetA>
    static __device__ inline f32x16 forward(GetA getA, const f32x16 (&cf)[2], const f32x16 (&b2)[2],
                                            const float (&s1)[kL1Slots32], float x0, float x1,
                                            float x2)
    {
        Frag B1[S::KS1];
#pragma unroll
        for (int ks = 0; ks < S::KS1; ks++)
            B1[ks] = frag_of(s1, ks);
        f32x16 a[2] = {cf[0], cf[1]};
        dense<2>(getA, S::FRAG_L1, B1, a);

        Frag B2[S::KS2];
        chain(a, B2);
        a[0] = b2[0];
        a[1] = b2[1];
        dense<2>(getA, S::FRAG_L2, B2, a);

        Frag B3[S::KS3];
        l3_frags(a, x0, x1, x2, B3);
        a[0] = f32x16{};
        a[1] = f32x16{};
        dense<2>(getA, S::FRAG_L3, B3, a);

        Frag B4[S::KS4];
        chain(a, B4);
        f32x16 y[2] = {f32x16{}, f32x16{}};
        dense<1>(getA, S::FRAG_L4, B4, y);
        return y[0];
    }
};

}  // namespace fab
