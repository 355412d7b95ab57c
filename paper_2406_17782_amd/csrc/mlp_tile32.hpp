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
//
// L4 (4 outputs) runs on 16x16x32 MFMA with the same B fragments: read as a
// 16x16x32 operand, lane l supplies K block l/16, so blocks 0 and 2 carry
// pixels 0..15 (lane groups 0 and 1) and blocks 1 and 3 pixels 16..31.  The
// packed A operand puts the four output rows of pixels 0..15 in rows 0..3
// (weights in K blocks 0 and 2) and those of pixels 16..31 in rows 4..7
// (K blocks 1 and 3); the 16x16 result layout then leaves output i of pixel
// l in register i of lane l for l < 32, and the layer's bias rides in the C
// operand.  Half the matrix work of a 32x32x16 L4 with 4 of 32 rows used.
//
// BF16 hidden layers are scaled per neuron by powers of two (chosen from
// bounds on their activations when the image is packed, undone by the next
// layer's weights) so that every activation lies below 1; the ReLU is then
// the [0, 1] clamp of the packed conversion to bf16, one instruction per two
// values.  Power-of-two scaling commutes with bf16 rounding and FP32
// accumulation, so the results are those of the unscaled network.
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
    static constexpr int FRAG_L4 = FRAG_L3 + 2 * KS3;    // 16x16x32 operands, one per k-step
    static constexpr int NFRAG = FRAG_L4 + KS4;          // 28
};

// Pack eight floats into a bf16 fragment, each pair with the [0, 1] clamp of
// v_cvt_pk_bf16_f32 (NaN -> 0): the ReLU of activations scaled below 1.
// The compiler does not emit this form, and its hazard checks do not look
// inside inline assembly, so the asm is kept safe by construction:
//  - its inputs are MFMA results, read only after `guard`, a compiler-visible
//    VALU read of the same MFMA result (the compiler makes that read wait
//    for the MFMA, which writes all its result registers at once), passed
//    as an input so that the asm cannot be scheduled before it;
//  - its outputs are early-clobber (no output overwrites a later input);
//  - it ends with two wait states, the gap a VALU write needs before an
//    MFMA reads the register as an operand.
__device__ inline bf16x8 cvt_clamp8(f32x8 v, float guard)
{
    unsigned w0, w1, w2, w3;
    asm("v_cvt_pk_bf16_f32 %0, %4, %5 clamp\n\t"
        "v_cvt_pk_bf16_f32 %1, %6, %7 clamp\n\t"
        "v_cvt_pk_bf16_f32 %2, %8, %9 clamp\n\t"
        "v_cvt_pk_bf16_f32 %3, %10, %11 clamp\n\t"
        "s_nop 1"
        : "=&v"(w0), "=&v"(w1), "=&v"(w2), "=&v"(w3)
        : "v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3]), "v"(v[4]), "v"(v[5]), "v"(v[6]),
          "v"(v[7]), "v"(guard));
    return __builtin_bit_cast(bf16x8, (u32x4){w0, w1, w2, w3});
}

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
// then L2's bias [64] (scaled; the C operand's rows), the L4 C operand
// [64 lanes][4] (16x16 layout: the four biases in lanes 0..31), the hidden
// neurons' scale exponents [3 layers][64] (int32) and the scales of the
// per-fabric first-layer biases c_f [64] (float, 2^-e).
template <int P> struct Tile32 {
    using M = Mfma<P>;
    using Frag = typename M::Frag;
    using S = DecShape32<8>;
    using FM = FeatureMath<P>;
    // The ReLU by the clamp of the conversion (activations scaled below 1).
    static constexpr bool kClampRelu = P == FABRIC_BF16;

    // Rectified fragments ks = 0 .. 2 * NMB - 1 of the 16 x NMB chained
    // values in acc (fragments 2 mb and 2 mb + 1 come from acc[mb]).
    template <int NMB, int KS>
    static __device__ inline void relu_frags(const f32x16 (&acc)[2], Frag (&B)[KS])
    {
#pragma unroll
        for (int mb = 0; mb < NMB; mb++) {
            if constexpr (kClampRelu) {
                // Element 0 clamped by the compiler: the guard of this MFMA result.
                const float g = __builtin_amdgcn_fmed3f(acc[mb][0], 0.0f, 1.0f);
                f32x8 lo, hi;
#pragma unroll
                for (int j = 0; j < 8; j++) {
                    lo[j] = acc[mb][j];
                    hi[j] = acc[mb][8 + j];
                }
                lo[0] = g;
                B[2 * mb] = cvt_clamp8(lo, g);
                B[2 * mb + 1] = cvt_clamp8(hi, g);
            } else {
                float v[16];
#pragma unroll
                for (int j = 0; j < 16; j++)
                    v[j] = acc[mb][j];
                B[2 * mb] = M::relu(frag_of(v, 0));
                B[2 * mb + 1] = M::relu(frag_of(v, 1));
            }
        }
    }

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
        // The phase in revolutions: the coordinate less whole periods, over the
        // period.  sin and cos are periodic, so the reduction only keeps the
        // argument small; it need not land exactly in [0, period).
        const float c = g ? v : u;
        const float ph = fmaf(-per, floorf(c * iper), c) * iper;
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
        // Bin b: exp(-d^2 / 2) with d = 8 tau - (4 g + b) - 1/2, the scale of
        // gauss_q folded into one FMA from tau.
        constexpr float q = FM::kGaussQ;
#pragma unroll
        for (int b = 0; b < 4; b++)
            s1[16 + b] = FM::gauss_q(fmaf(tau, 8.0f * q, -q * ((float)(4 * g + b) + 0.5f)));
    }

    template <int KS>
    static __device__ inline void chain(const f32x16 (&acc)[2], Frag (&B)[KS])
    {
        relu_frags<2>(acc, B);
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
        relu_frags<2>(a, B3);
        const float v[3] = {x0, x1, x2};
        B3[4] = frag_of(v, 0);
    }

    // Forward: cf / b2 / b4 are the C operands of L1, L2 (per lane, both
    // M-blocks) and L4 (16x16 layout).  Returns the four outputs, bias
    // included, in registers 0..3 of lanes 0..31 (output i of pixel l in
    // lane l).
    template <typename GetA>
    static __device__ inline f32x4 forward(GetA getA, const f32x16 (&cf)[2], const f32x16 (&b2)[2],
                                           f32x4 b4, const float (&s1)[kL1Slots32], float x0,
                                           float x1, float x2)
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
        f32x4 y = b4;
#pragma unroll
        for (int ks = 0; ks < S::KS4; ks++)
            y = M::mma(getA(S::FRAG_L4 + ks), B4[ks], y);
        return y;
    }
};

}  // namespace fab
