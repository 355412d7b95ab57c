// Decoder tile of 32 pixels with OCP FP8-E4M3 operands on the scaled
// 32x32x64 MFMA (v_mfma_scale_f32_32x32x64_f8f6f4), FP32 accumulation.
//
// Per-layer scales are powers of two carried by the instruction's E8M0 scale
// operands.  Layer l stores its weights as W * 2^eW[l] and takes its input as
// h * 2^ein[l]; the A-scale 2^(eout[l] - eW[l]) and B-scale 2^(-ein[l]) make
// the accumulator come out as 2^eout[l] * (W h + b) (the C-operand biases are
// stored pre-scaled), which is the next layer's input scale:
// ein = {kFeatExp, eh1, eh2, eh3}, eout = {eh1, eh2, eh3, 0}.  The hidden
// exponents come from activation maxima measured on a calibration batch, the
// weight exponents from each layer's largest weight.  Hidden activations are
// clamped to [0, 448] (ReLU and E4M3 saturation in one v_med3) before
// rounding to E4M3 (round to nearest even).
//
// Operand layout: lane group g = l/32 of lane l holds bytes j = 0..31 of its
// row (A) or column (B); A and B use the same byte order, so the contraction
// pairs A's byte (g, j) with B's byte (g, j) whatever K index the hardware
// gives it.  Byte (g, j) of a chained layer carries neuron chain32_neuron(g, j)
// -- exactly the 32 accumulator values the lane group holds after a 32x32
// layer -- so layers chain without data movement, as in mlp_tile32.hpp.
//   L1: one k-step: bytes 0..19 the spatial slots of mlp_tile32.hpp, rest 0
//   L2: one k-step of chained neurons
//   L3: one k-step of chained neurons, then L3's three angular inputs and
//       bias on one 32x32x16 BF16 MFMA into the same accumulators (slots
//       0..2 of lane group g: g = 0 wi.x, wi.y, wi.z; g = 1 wo.x, wo.y and
//       the constant 1 carrying the bias), its weights stored as
//       2^eh3 W in BF16: a 64-deep FP8 step for three inputs would cost
//       twice the matrix cycles.
//   L4: one 16x16x128 FP8 MFMA reading L4's chained B operand as is: lane l
//       supplies K block l/16, so blocks 0 and 2 carry pixels 0..15 (lane
//       groups 0 and 1) and blocks 1 and 3 pixels 16..31; the A operand
//       holds the four output rows of pixels 0..15 in rows 0..3 (weights in
//       K blocks 0 and 2) and those of pixels 16..31 in rows 4..7 (K blocks 1
//       and 3), which leaves output i of pixel l in register i of lane l for
//       l < 32 -- half the cycles of a 32x32x64 step with 4 of 32 rows used.
#pragma once

#include "mlp_tile32.hpp"

namespace fab {

typedef int i32x8 __attribute__((ext_vector_type(8)));

// A fragments of the FP8 image (64 lanes x 32 bytes each), then L3's
// angular BF16 fragments (64 lanes x 16 bytes, one per M-block).
struct DecShapeF8 {
    static constexpr int FRAG_L1 = 0;    // 2 M-blocks x 1 k-step
    static constexpr int FRAG_L2 = 2;    // 2 x 1
    static constexpr int FRAG_L3 = 4;    // 2 x 1 (chained neurons)
    static constexpr int FRAG_L4 = 6;    // one 16x16x128 operand
    static constexpr int NFRAG = 7;
    static constexpr int NANG = 2;       // BF16 angular fragments of L3
};

// Features and directions enter unscaled: they lie in [-1, 1], where E4M3
// keeps full relative precision down to 2^-6 and absolute precision 2^-10
// below.
constexpr int kFeatExp = 0;
constexpr float kF8Max = 448.0f;     // largest finite E4M3 value

// Scales of a packed FP8 decoder (stored in its image after the biases).
struct F8Header {
    int sa[4];         // E8M0 A-scale per layer: 127 + eout - eW
    int sb[4];         // E8M0 B-scale per layer: 127 - ein
    int unused;
    float cf_mult;     // 2^eh1, applied to c_f when it is staged
    float hmax[3];     // calibrated maxima of h1, h2, h3
    float wmax[4];     // largest |weight| per layer
    int eh[3];         // hidden exponents
    int ew[4];         // weight exponents
    int pad[8];
};
static_assert(sizeof(F8Header) == 128, "header size");

// Round the first NV of 32 floats (already scaled, within +-448) to E4M3
// bytes, element j at byte j; bytes NV..31 are zero.  Each word is written as
// two 16-bit halves; the first conversion's `old` operand (the half it keeps)
// is overwritten by the second, so any register serves and none has to be
// zeroed.
template <int NV = 32> __device__ inline i32x8 pack_f8x32(const float (&v)[32])
{
    i32x8 w;
#pragma unroll
    for (int q = 0; q < 8; q++) {
        if (4 * q >= NV) {
            w[q] = 0;
            continue;
        }
        const int lo = __builtin_amdgcn_cvt_pk_fp8_f32(v[4 * q], v[4 * q + 1],
                                                       __builtin_bit_cast(int, v[4 * q]), false);
        w[q] = 4 * q + 2 < NV ? __builtin_amdgcn_cvt_pk_fp8_f32(v[4 * q + 2], v[4 * q + 3], lo, true)
                              : (lo & 0xFFFF);
    }
    return w;
}

struct TileF8 {
    static __device__ inline f32x16 mma(i32x8 a, i32x8 b, f32x16 c, int sa, int sb)
    {
        // cbsz = blgp = 0: both operands E4M3; scales from byte 0 of sa / sb.
        return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, sa, 0, sb);
    }
    static __device__ inline f32x4 mma16(i32x8 a, i32x8 b, f32x4 c, int sa, int sb)
    {
        return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, sa, 0, sb);
    }

    // Rectify, clamp to the E4M3 range and round a layer's accumulators into
    // the next layer's B operand.
    static __device__ inline i32x8 chain(const f32x16 (&acc)[2])
    {
        float v[32];
#pragma unroll
        for (int c = 0; c < 32; c++)
            v[c] = __builtin_amdgcn_fmed3f(acc[c >> 4][c & 15], 0.0f, kF8Max);
        return pack_f8x32(v);
    }

    // The B operands of L1 (the 20 spatial slots) and of L3's angular BF16
    // step (three inputs, slots 0..2) of one tile.
    static __device__ inline i32x8 l1_operand(const float (&s1)[kL1Slots32])
    {
        float v[32];
#pragma unroll
        for (int c = 0; c < 32; c++)
            v[c] = c < kL1Slots32 ? s1[c] : 0.0f;
        return pack_f8x32<kL1Slots32>(v);
    }
    static __device__ inline bf16x8 l3x_frag(float x0, float x1, float x2)
    {
        const f32x8 v = {x0, x1, x2, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        return Mfma<FABRIC_BF16>::from8(v);
    }

    // Two independent tiles, layer by layer in alternation, so that one
    // tile's MFMAs run while the other's activations are rounded.  a0 / a1
    // hold each tile's L1 C operand (2^eh1 c_f) on entry and W4 h3 (outputs
    // 0..3 of pixel l in registers 0..3 of lane l < 32) on exit; getB2(mb)
    // is L2's (shared) C operand, A3x L3's angular BF16 fragments.
    template <typename GetA, typename GetB2>
    static __device__ inline void forward2(GetA getA, const F8Header &h, f32x16 (&a0)[2],
                                           f32x16 (&a1)[2], GetB2 getB2,
                                           const bf16x8 (&A3x)[DecShapeF8::NANG], i32x8 B1a,
                                           i32x8 B1b, bf16x8 xa, bf16x8 xb)
    {
#pragma unroll
        for (int mb = 0; mb < 2; mb++)
            a0[mb] = mma(getA(DecShapeF8::FRAG_L1 + mb), B1a, a0[mb], h.sa[0], h.sb[0]);
#pragma unroll
        for (int mb = 0; mb < 2; mb++)
            a1[mb] = mma(getA(DecShapeF8::FRAG_L1 + mb), B1b, a1[mb], h.sa[0], h.sb[0]);

        const i32x8 B2a = chain(a0);
#pragma unroll
        for (int mb = 0; mb < 2; mb++)
            a0[mb] = mma(getA(DecShapeF8::FRAG_L2 + mb), B2a, getB2(mb), h.sa[1], h.sb[1]);
        const i32x8 B2b = chain(a1);
#pragma unroll
        for (int mb = 0; mb < 2; mb++)
            a1[mb] = mma(getA(DecShapeF8::FRAG_L2 + mb), B2b, getB2(mb), h.sa[1], h.sb[1]);

        const i32x8 B3a = chain(a0);
#pragma unroll
        for (int mb = 0; mb < 2; mb++) {
            a0[mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A3x[mb], xa, f32x16{}, 0, 0, 0);
            a0[mb] = mma(getA(DecShapeF8::FRAG_L3 + mb), B3a, a0[mb], h.sa[2], h.sb[2]);
        }
        const i32x8 B3b = chain(a1);
#pragma unroll
        for (int mb = 0; mb < 2; mb++) {
            a1[mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A3x[mb], xb, f32x16{}, 0, 0, 0);
            a1[mb] = mma(getA(DecShapeF8::FRAG_L3 + mb), B3b, a1[mb], h.sa[2], h.sb[2]);
        }

        const i32x8 B4a = chain(a0);
        const f32x4 ya = mma16(getA(DecShapeF8::FRAG_L4), B4a, f32x4{}, h.sa[3], h.sb[3]);
        const i32x8 B4b = chain(a1);
        const f32x4 yb = mma16(getA(DecShapeF8::FRAG_L4), B4b, f32x4{}, h.sa[3], h.sb[3]);
        // The scaled MFMA builtins are not marked convergent, so the compiler
        // would otherwise sink the whole chain into a caller's lane-divergent
        // branch (e.g. the store of lane group 0), where lanes with EXEC off
        // never build their share of the B operands.  An opaque use of both
        // results in every lane pins the chain to uniform control flow.
        float t0 = ya[0], t1 = ya[1], t2 = ya[2], t3 = ya[3];
        float u0 = yb[0], u1 = yb[1], u2 = yb[2], u3 = yb[3];
        asm volatile("" : "+v"(t0), "+v"(t1), "+v"(t2), "+v"(t3), "+v"(u0), "+v"(u1), "+v"(u2),
                     "+v"(u3));
        a0[0][0] = t0;
        a0[0][1] = t1;
        a0[0][2] = t2;
        a0[0][3] = t3;
        a1[0][0] = u0;
        a1[0][1] = u1;
        a1[0][2] = u2;
        a1[0][3] = u3;
    }
};

}  // namespace fab
