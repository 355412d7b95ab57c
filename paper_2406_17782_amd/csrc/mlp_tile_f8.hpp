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
//   L2, L4: one k-step of chained neurons
//   L3: k-step 0 chained neurons; k-step 1 bytes 0..2: g = 0 (wi.x, wi.y,
//       wi.z), g = 1 (wo.x, wo.y, 1), the constant carrying the layer's bias
#pragma once

#include "mlp_tile32.hpp"

namespace fab {

typedef int i32x8 __attribute__((ext_vector_type(8)));

// A fragments of the FP8 image (64 lanes x 32 bytes each).
struct DecShapeF8 {
    static constexpr int FRAG_L1 = 0;    // 2 M-blocks x 1 k-step
    static constexpr int FRAG_L2 = 2;    // 2 x 1
    static constexpr int FRAG_L3 = 4;    // 2 x 2 (mb-major)
    static constexpr int FRAG_L4 = 8;    // 1 x 1 (rows 0..3)
    static constexpr int NFRAG = 9;
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
    int sb_ang;        // E8M0 B-scale of L3's angular k-step: 127 - kFeatExp
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

    // Forward of one tile.  cf: L1 C operand (2^eh1 c_f rows of this lane),
    // b2: L2's (pre-scaled).  s1: the 20 spatial slots, x: the three L3 extra
    // inputs of this lane group.  Returns W4 h3 (without its bias) in
    // accumulator registers 0..3 of lane group 0.
    template <typename GetA>
    static __device__ inline f32x16 forward(GetA getA, const F8Header &h, const f32x16 (&cf)[2],
                                            const f32x16 (&b2)[2], const float (&s1)[kL1Slots32],
                                            float x0, float x1, float x2)
    {
        static_assert(kFeatExp == 0, "features enter unscaled");
        float v[32];
#pragma unroll
        for (int c = 0; c < 32; c++)
            v[c] = c < kL1Slots32 ? s1[c] : 0.0f;
        const i32x8 B1 = pack_f8x32<kL1Slots32>(v);
        f32x16 a[2] = {cf[0], cf[1]};
#pragma unroll
        for (int mb = 0; mb < 2; mb++)
            a[mb] = mma(getA(DecShapeF8::FRAG_L1 + mb), B1, a[mb], h.sa[0], h.sb[0]);

        const i32x8 B2 = chain(a);
        a[0] = b2[0];
        a[1] = b2[1];
#pragma unroll
        for (int mb = 0; mb < 2; mb++)
            a[mb] = mma(getA(DecShapeF8::FRAG_L2 + mb), B2, a[mb], h.sa[1], h.sb[1]);

        const i32x8 B3 = chain(a);
#pragma unroll
        for (int c = 0; c < 32; c++)
            v[c] = 0.0f;
        v[0] = x0;
        v[1] = x1;
        v[2] = x2;
        const i32x8 B3x = pack_f8x32<3>(v);
#pragma unroll
        for (int mb = 0; mb < 2; mb++) {
            a[mb] = mma(getA(DecShapeF8::FRAG_L3 + 2 * mb), B3, f32x16{}, h.sa[2], h.sb[2]);
            a[mb] = mma(getA(DecShapeF8::FRAG_L3 + 2 * mb + 1), B3x, a[mb], h.sa[2], h.sb_ang);
        }

        const i32x8 B4 = chain(a);
        f32x16 y = mma(getA(DecShapeF8::FRAG_L4), B4, f32x16{}, h.sa[3], h.sb[3]);
        // The scaled MFMA builtin is not marked convergent, so the compiler
        // would otherwise sink the whole chain into a caller's lane-divergent
        // branch (e.g. the store of lane group 0), where lanes with EXEC off
        // never build their share of the B operands.  An opaque use of the
        // result in every lane pins the chain to uniform control flow.
        float y0 = y[0], y1 = y[1], y2 = y[2], y3 = y[3];
        asm volatile("" : "+v"(y0), "+v"(y1), "+v"(y2), "+v"(y3));
        y[0] = y0;
        y[1] = y1;
        y[2] = y2;
        y[3] = y3;
        return y;
    }

    // The B operands of L1 (the 20 spatial slots) and of L3's angular k-step
    // (three inputs: word 0 only) of one tile.
    static __device__ inline i32x8 l1_operand(const float (&s1)[kL1Slots32])
    {
        float v[32];
#pragma unroll
        for (int c = 0; c < 32; c++)
            v[c] = c < kL1Slots32 ? s1[c] : 0.0f;
        return pack_f8x32<kL1Slots32>(v);
    }
    static __device__ inline int l3x_word(float x0, float x1, float x2)
    {
        const int lo = __builtin_amdgcn_cvt_pk_fp8_f32(x0, x1, __builtin_bit_cast(int, x0), false);
        return __builtin_amdgcn_cvt_pk_fp8_f32(x2, 0.0f, lo, true);
    }

    // Two independent tiles, layer by layer in alternation, so that one
    // tile's MFMAs run while the other's activations are rounded.  a0 / a1
    // hold each tile's L1 C operand (2^eh1 c_f) on entry and W4 h3 (rows
    // 0..3 in lane group 0) on exit; getB2(mb) is L2's (shared) C operand.
    template <typename GetA, typename GetB2>
    static __device__ inline void forward2(GetA getA, const F8Header &h, f32x16 (&a0)[2],
                                           f32x16 (&a1)[2], GetB2 getB2, i32x8 B1a, i32x8 B1b,
                                           int xa, int xb)
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
        const i32x8 B3xa = i32x8{xa, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int mb = 0; mb < 2; mb++) {
            a0[mb] = mma(getA(DecShapeF8::FRAG_L3 + 2 * mb), B3a, f32x16{}, h.sa[2], h.sb[2]);
            a0[mb] = mma(getA(DecShapeF8::FRAG_L3 + 2 * mb + 1), B3xa, a0[mb], h.sa[2], h.sb_ang);
        }
        const i32x8 B3b = chain(a1);
        const i32x8 B3xb = i32x8{xb, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int mb = 0; mb < 2; mb++) {
            a1[mb] = mma(getA(DecShapeF8::FRAG_L3 + 2 * mb), B3b, f32x16{}, h.sa[2], h.sb[2]);
            a1[mb] = mma(getA(DecShapeF8::FRAG_L3 + 2 * mb + 1), B3xb, a1[mb], h.sa[2], h.sb_ang);
        }

        const i32x8 B4a = chain(a0);
        a0[0] = mma(getA(DecShapeF8::FRAG_L4), B4a, f32x16{}, h.sa[3], h.sb[3]);
        const i32x8 B4b = chain(a1);
        a1[0] = mma(getA(DecShapeF8::FRAG_L4), B4b, f32x16{}, h.sa[3], h.sb[3]);
        // Pin both results to uniform control flow (see forward).
        float t0 = a0[0][0], t1 = a0[0][1], t2 = a0[0][2], t3 = a0[0][3];
        float u0 = a1[0][0], u1 = a1[0][1], u2 = a1[0][2], u3 = a1[0][3];
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
