// Per-wavefront decoder tile: 16 pixels (N) through the dense layers on MFMA.
// Shared by the shading kernel and the training kernel so that both compute
// the forward pass with identical arithmetic.
#pragma once

#include "common.hpp"
#include "model.hpp"

namespace fab {

// Transcendentals of the decoder's input encoding and output decoding.
// Low-precision operands (bf16, fp16): hardware sine/cosine (argument in
// revolutions) at the base frequency and angle doubling for the next three
// (the doubled phase error, 8 x 2^-22, is far below the operand rounding),
// hardware exp2/log2.
template <int P> struct FeatureMath {
    static constexpr bool kDoubling = true;
    static __device__ inline void sincos2pi(float x, float *s, float *c)
    {
        *s = __builtin_amdgcn_sinf(x);
        *c = __builtin_amdgcn_cosf(x);
    }
    static __device__ inline float log2(float x) { return __builtin_amdgcn_logf(x); }
    // exp(-d^2 / 2)
    static __device__ inline float gauss(float d)
    {
        return __builtin_amdgcn_exp2f(-0.72134752044448170368f * d * d);
    }
    // exp(-d^2 / 2) from qd = kGaussQ d: exp2(-(qd)^2), kGaussQ^2 = log2(e) / 2
    static constexpr float kGaussQ = 0.84932180028801904f;
    static __device__ inline float gauss_q(float qd) { return __builtin_amdgcn_exp2f(-(qd * qd)); }
    // e^y - 1
    static __device__ inline float expm1(float y)
    {
        return __builtin_amdgcn_exp2f(1.44269504088896340736f * y) - 1.0f;
    }
};
// Reference precision: library functions, every frequency evaluated directly.
template <> struct FeatureMath<FABRIC_FP32> {
    static constexpr bool kDoubling = false;
    static __device__ inline void sincos2pi(float x, float *s, float *c)
    {
        sincospif(2.0f * x, s, c);
    }
    static __device__ inline float log2(float x) { return log2f(x); }
    static __device__ inline float gauss(float d) { return expf(-0.5f * d * d); }
    static constexpr float kGaussQ = 0.84932180028801904f;
    static __device__ inline float gauss_q(float qd) { return exp2f(-(qd * qd)); }
    static __device__ inline float expm1(float y) { return expm1f(y); }
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
        using FM = FeatureMath<P>;
        if (FM::kDoubling) {
            float x = ldexpf(coord, k0);
            float sn, cs;
            FM::sincos2pi(wrap_period(x, per, iper) * iper, &sn, &cs);
#pragma unroll
            for (int q = 0; q < 4; q++) {
                s1[q] = sn;
                s1[4 + q] = cs;
                const float s2 = 2.0f * sn * cs;           // sin 2t
                cs = fmaf(-2.0f * sn, sn, 1.0f);            // cos 2t
                sn = s2;
            }
        } else {
#pragma unroll
            for (int q = 0; q < 4; q++) {
                // frac(2^k coord / period): the power-of-two scaling is exact
                // and the reduction into the period is exact, leaving one rounding.
                float x = ldexpf(coord, k0 + q);
                float ph = wrap_period(x, per, iper) * iper;
                FM::sincos2pi(ph, &s1[q], &s1[4 + q]);
            }
        }
        // tau = clamp((log2 r + 14) / 16, 0, 1); bin b = exp(-((8 tau - b - 1/2)^2) / 2)
        float tau = fminf(fmaxf((FM::log2(r) + 14.0f) * (1.0f / 16.0f), 0.0f), 1.0f);
#pragma unroll
        for (int b2 = 0; b2 < 2; b2++) {
            float d = 8.0f * tau - (float)(2 * grp + b2) - 0.5f;
            s1[8 + b2] = FM::gauss(d);
        }
    }

    // Frag ks from slot values vals[ks*KPL .. ks*KPL + KPL - 1] (0 past NSL).
    template <int NSL>
    static __device__ inline Frag frag_of(const float (&vals)[NSL], int ks)
    {
        if constexpr (KPL == 1) {
            return ks < NSL ? vals[ks] : 0.0f;
        } else {
            f32x8 v;
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const int c = ks * 8 + j;
                v[j] = c < NSL ? vals[c] : 0.0f;
            }
            return M::from8(v);
        }
    }

    template <int NSL, int KS>
    static __device__ inline void to_frags(const float (&vals)[NSL], Frag (&B)[KS])
    {
#pragma unroll
        for (int ks = 0; ks < KS; ks++)
            B[ks] = frag_of(vals, ks);
    }

    // The 16 chained slot values of a layer output, in slot order.
    static __device__ inline void chain_vals(const f32x4 (&acc)[4], float (&v)[kChainSlots])
    {
#pragma unroll
        for (int c = 0; c < kChainSlots; c++)
            v[c] = acc[c >> 2][c & 3];
    }

    // Chained slots of a layer output: slot c <- acc[c/4][c%4] (optionally ReLU).
    template <int KS>
    static __device__ inline void chain(const f32x4 (&acc)[4], bool relu, Frag (&B)[KS])
    {
        float v[kChainSlots];
        chain_vals(acc, v);
#pragma unroll
        for (int ks = 0; ks < KS; ks++) {
            B[ks] = frag_of(v, ks);
            if (relu)
                B[ks] = M::relu(B[ks]);   // after rounding: same result, packed
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

        // L3 slots: 16 chained neurons (rectified) then the angular inputs
        // (not rectified); the chained k-steps take the packed ReLU.
        Frag B3[S::KS3];
        {
            float v[kL3Slots];
#pragma unroll
            for (int c = 0; c < kChainSlots; c++)
                v[c] = a2[c >> 2][c & 3];
            v[kChainSlots] = ang0;
            v[kChainSlots + 1] = ang1;
            static_assert(kChainSlots % KPL == 0, "chained slots fill whole k-steps");
#pragma unroll
            for (int ks = 0; ks < S::KS3; ks++) {
                B3[ks] = frag_of(v, ks);
                if ((ks + 1) * KPL <= kChainSlots)
                    B3[ks] = M::relu(B3[ks]);
            }
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
