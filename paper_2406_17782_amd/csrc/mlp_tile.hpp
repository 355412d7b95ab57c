// Per-wavefront decoder tile: 16 pixels (N) through the dense layers on MFMA.
// Shared by the shading kernel and the training kernel so that both compute
// the forward pass with identical arithmetic.
#pragma once

#include "common.hpp"
#include "model.hpp"

namespace fab {

template <int P> struct FeatureMath {
    // Low-precision operands: the hardware sine/cosine (argument in
    // revolutions) are far more accurate than the operands' rounding.
    static __device__ inline void sincos2pi(float x, float *s, float *c)
    {
        *s = __builtin_amdgcn_sinf(x);
        *c = __builtin_amdgcn_cosf(x);
    }
};
// Reference precision: correctly rounded-range sin/cos of 2 pi x.
template <> struct FeatureMath<FABRIC_FP32> {
    static __device__ inline void sincos2pi(float x, float *s, float *c)
    {
        sincospif(2.0f * x, s, c);
    }
};

template <int P> struct Tile {
    using M = Mfma<P>;
    using Frag = typename M::Frag;
    using S = DecShape<M::KPL>;
    static constexpr int KPL = M::KPL;
    static constexpr int NS1 = S::KS1 * KPL;

    // L1 slot values of lane group `grp` for its pixel (see common.hpp):
    // 4 sines and 4 cosines of the pattern-tiled position along u (groups 0,1)
    // or v (groups 2,3) at frequencies 2^k0..2^(k0+3), then one-blob bins
    // 2*grp and 2*grp+1 of the footprint size.
    static __device__ inline void spatial_slots(float u, float v, float r, float fwx, float fwy,
                                                float iwx, float iwy, int grp, float (&s1)[NS1])
    {
#pragma unroll
        for (int c = 0; c < NS1; c++)
            s1[c] = 0.0f;
        const bool axis_v = grp >= 2;
        const float per = axis_v ? fwy : fwx;
        const float iper = axis_v ? iwy : iwx;
        // Reduce into the period first so that the scaled value stays finite.
        const float coord = wrap_period(axis_v ? v : u, per, iper);
        const int k0 = 4 * (grp & 1);
#pragma unroll
        for (int q = 0; q < 4; q++) {
            // frac(2^k coord / period): the power-of-two scaling is exact and
            // the reduction into the period is exact, leaving one rounding.
            float x = ldexpf(coord, k0 + q);
            float ph = wrap_period(x, per, iper) * iper;
            FeatureMath<P>::sincos2pi(ph, &s1[q], &s1[4 + q]);
        }
        // tau = clamp((log2 r + 14) / 16, 0, 1); bin b = exp(-((8 tau - b - 1/2)^2) / 2)
        float tau = fminf(fmaxf((log2f(r) + 14.0f) * (1.0f / 16.0f), 0.0f), 1.0f);
#pragma unroll
        for (int b2 = 0; b2 < 2; b2++) {
            float d = 8.0f * tau - (float)(2 * grp + b2) - 0.5f;
            s1[8 + b2] = expf(-0.5f * d * d);
        }
    }

    template <int NSL, int KS>
    static __device__ inline void to_frags(const float (&vals)[NSL], Frag (&B)[KS])
    {
#pragma unroll
        for (int ks = 0; ks < KS; ks++)
#pragma unroll
            for (int j = 0; j < KPL; j++) {
                const int c = ks * KPL + j;
                M::set(B[ks], j, c < NSL ? vals[c] : 0.0f);
            }
    }

    // Chained slots of a layer output: slot c <- acc[c/4][c%4] (optionally ReLU).
    template <int KS>
    static __device__ inline void chain(const f32x4 (&acc)[4], bool relu, Frag (&B)[KS])
    {
#pragma unroll
        for (int ks = 0; ks < KS; ks++)
#pragma unroll
            for (int j = 0; j < KPL; j++) {
                const int c = ks * KPL + j;
                float val = 0.0f;
                if (c < kChainSlots)
                    val = relu ? fmaxf(acc[c >> 2][c & 3], 0.0f) : acc[c >> 2][c & 3];
                M::set(B[ks], j, val);
            }
    }

    // acc[mb] += sum_ks A(base + mb*KS + ks) * B[ks] for mb < NMB.
    template <int NMB, int KS, typename GetA>
    static __device__ inline void dense(GetA getA, int base, const Frag (&B)[KS], f32x4 (&acc)[4])
    {
#pragma unroll
        for (int mb = 0; mb < NMB; mb++)
#pragma unroll
            for (int ks = 0; ks < KS; ks++)
                acc[mb] = M::mma(getA(base + mb * KS + ks), B[ks], acc[mb]);
    }

    // Forward through all four layers.  cf: this lane's 16 first-layer biases
    // (c_f rows 16 mb + 4 grp + i); bias(q): C-operand biases of L2..L4.
    // Outputs the pre-activations of L1..L3 and y (rows 0..3 in lane group 0).
    template <typename GetA, typename GetBias>
    static __device__ inline void forward(GetA getA, GetBias bias, const f32x4 (&cf)[4],
                                          const float (&s1)[NS1], float ang0, float ang1,
                                          f32x4 (&a1)[4], f32x4 (&a2)[4], f32x4 (&a3)[4],
                                          f32x4 &y)
    {
        Frag B1[S::KS1];
        to_frags(s1, B1);
#pragma unroll
        for (int mb = 0; mb < 4; mb++)
            a1[mb] = cf[mb];
        dense<4>(getA, S::FRAG_L1, B1, a1);

        Frag B2[S::KS2];
        chain(a1, true, B2);
#pragma unroll
        for (int mb = 0; mb < 4; mb++)
            a2[mb] = bias(mb);
        dense<4>(getA, S::FRAG_L2, B2, a2);

        Frag B3[S::KS3];
#pragma unroll
        for (int ks = 0; ks < S::KS3; ks++)
#pragma unroll
            for (int j = 0; j < KPL; j++) {
                const int c = ks * KPL + j;
                float val = 0.0f;
                if (c < kChainSlots) val = fmaxf(a2[c >> 2][c & 3], 0.0f);
                else if (c == kChainSlots) val = ang0;
                else if (c == kChainSlots + 1) val = ang1;
                M::set(B3[ks], j, val);
            }
#pragma unroll
        for (int mb = 0; mb < 4; mb++)
            a3[mb] = bias(4 + mb);
        dense<4>(getA, S::FRAG_L3, B3, a3);

        Frag B4[S::KS4];
        chain(a3, true, B4);
        f32x4 y4[4];
        y4[0] = bias(8);
        dense<1>(getA, S::FRAG_L4, B4, y4);
        y = y4[0];
    }
};

// Angular inputs carried by lane group grp in L3 slots 16 and 17.
__device__ inline void angular_slots(int grp, float3 wi, float3 wo, float *ang0, float *ang1)
{
    *ang0 = grp == 0 ? wi.x : (grp == 1 ? wi.z : (grp == 2 ? wo.y : 0.0f));
    *ang1 = grp == 0 ? wi.y : (grp == 1 ? wo.x : 0.0f);
}

}  // namespace fab
