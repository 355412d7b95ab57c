// Shared device-side definitions of the gfx950 fabric library: the per-fabric
// table the kernels read, the MFMA operand traits per precision and the
// convention that maps a lane's operand slots to decoder inputs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fabric.h"

namespace fab {

constexpr float kPi = 3.14159265358979323846f;
// Cross-section slope limit of the yarn profile (radians).
constexpr float kThetaMax = kPi / 3.0f;
// k of the specular log mapping g(x) = ln(k x + 1) (Eq. (9), reflection).
constexpr float kSpec = 100.0f;
// Optical depth T*rho of the fabric's specular layer (Sec. 3.1).
constexpr float kTRho = 2.0f;

constexpr int kLatent = 32;
constexpr int kHid = 64;
constexpr int kFeat = 40;
constexpr int kEncIn = 524;
constexpr int kEncHid = 128;

// Decoder parameter offsets inside the flat FP32 vector (rows = outputs).
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + 64 * 72;
constexpr int kOffW2 = kOffB1 + 64;
constexpr int kOffB2 = kOffW2 + 64 * 64;
constexpr int kOffW3 = kOffB2 + 64;
constexpr int kOffB3 = kOffW3 + 64 * 69;
constexpr int kOffW4 = kOffB3 + 64;
constexpr int kOffB4 = kOffW4 + 4 * 64;
constexpr int kNDec = kOffB4 + 4;
static_assert(kNDec == FABRIC_N_DECODER_PARAMS, "decoder layout");
// Encoder offsets relative to the start of the encoder block.
constexpr int kOffE1 = 0;
constexpr int kOffC1 = kOffE1 + kEncHid * kEncIn;
constexpr int kOffE2 = kOffC1 + kEncHid;
constexpr int kOffC2 = kOffE2 + kEncHid * kEncHid;
constexpr int kOffE3 = kOffC2 + kEncHid;
constexpr int kOffC3 = kOffE3 + kEncHid * kEncHid;
constexpr int kOffE4 = kOffC3 + kEncHid;
constexpr int kOffC4 = kOffE4 + kLatent * kEncHid;
constexpr int kNEnc = kOffC4 + kLatent;
static_assert(kNEnc == FABRIC_N_ENCODER_PARAMS, "encoder layout");

enum Yarn : int { kWarp = 0, kWeft = 1, kHole = 2 };

// Per-fabric constants as the kernels read them.  `cell` packs, per cell
// (i, j) at [j * 16 + i]: bit 15 = warp on top; bits 0-4 = offset of the cell
// inside the float (run of cells with the same yarn on top) of that top yarn;
// bits 5-9 = run length, 0 when the yarn never goes under (no along tilt).
struct alignas(16) DevFabric {
    int32_t wx, wy;
    float fwx, fwy, inv_wx, inv_wy;
    float alpha[2];
    float alpha2m1[2];       // 1 - alpha^2
    float ia2m1[2];          // 1/alpha^2 - 1
    float inv_pi_alpha[2];   // 1 / (pi alpha)
    float beta[2], incl[2];
    float cos_twist[2], sin_twist[2];
    float half_width[2], inv_half_width[2];   // (1 - gap)/2 and its inverse
    float wblend[2];
    float kd[2][3], ks[2][3];
    uint16_t cell[256];
};

// Inter-yarn visibility (V of Eq. (3)-(4)): per fabric, the tabulated height
// field of one pattern period, kVisRes texels per cell and axis, row-major
// (tw = wx kVisRes columns, th = wy kVisRes rows) at texel offset `off` of
// the shared table, and its largest texel.
constexpr int kVisRes = 16;
constexpr int kVisSteps = 32;   // march length in texel steps: two cells
struct VisFabric {
    int32_t off, tw, th;
    float hmax;
};
// tex == nullptr: V = 1 everywhere.
struct VisArgs {
    const float *tex;
    const VisFabric *fab;
};

// ---------------------------------------------------------------------------
// MFMA operand traits.  All variants are 16 x 16 output tiles in the
// "transposed" orientation: M = output neurons, N = 16 pixels, K = inputs.
// Per the CDNA 16x16xK layout, lane l holds A[m = l%16][k = KPL*(l/16) + j],
// B[k = KPL*(l/16) + j][n = l%16] and D[m = 4*(l/16) + i][n = l%16].
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// Compensated (Kahan) FP32 sum, for the fixed-order reductions of the
// training kernels: the error stays at a few units of the last place of the
// sum of magnitudes, independent of the number of terms.
struct KahanSum {
    float s = 0.0f, c = 0.0f;
    __device__ inline void add(float x)
    {
        const float y = x - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ inline float value() const { return s - c; }
};

template <int P> struct Mfma;

template <> struct Mfma<FABRIC_FP32> {
    static constexpr int KPL = 1;            // K values per lane per step
    using Frag = float;
    static __device__ inline f32x4 mma(Frag a, Frag b, f32x4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ inline void set(Frag &f, int j, float v) { (void)j; f = v; }
    static __device__ inline Frag zero() { return 0.0f; }
    static __device__ inline Frag relu(Frag f) { return fmaxf(f, 0.0f); }
};

// ReLU of eight 16-bit floats at once: for both bf16 and fp16 a value is
// negative exactly when its bit pattern is a negative int16, so a packed
// signed-integer max against 0 clamps it (-0 becomes +0).
typedef short s16x8 __attribute__((ext_vector_type(8)));
template <typename F> __device__ inline F relu16x8(F f)
{
    s16x8 s = __builtin_bit_cast(s16x8, f);
    s = __builtin_elementwise_max(s, (s16x8)(0));
    return __builtin_bit_cast(F, s);
}

typedef float f32x8 __attribute__((ext_vector_type(8)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// Eight floats rounded pairwise into one 8 x 16-bit fragment (H2 = the
// matching 2-wide 16-bit vector): one packed conversion per pair.
template <typename F, typename H2> __device__ inline F pack8(f32x8 v)
{
    u32x4 w;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        H2 h = __builtin_convertvector((f32x2){v[2 * q], v[2 * q + 1]}, H2);
        w[q] = __builtin_bit_cast(unsigned, h);
    }
    return __builtin_bit_cast(F, w);
}
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

template <> struct Mfma<FABRIC_BF16> {
    static constexpr int KPL = 8;
    using Frag = bf16x8;
    static __device__ inline f32x4 mma(Frag a, Frag b, f32x4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    static __device__ inline void set(Frag &f, int j, float v) { f[j] = (__bf16)v; }
    static __device__ inline Frag relu(Frag f) { return relu16x8(f); }
    // Round eight floats at once (pairs map onto packed conversions).
    static __device__ inline Frag from8(f32x8 v) { return pack8<Frag, bf16x2>(v); }
    static __device__ inline Frag zero()
    {
        Frag f;
        for (int j = 0; j < 8; j++) f[j] = (__bf16)0.0f;
        return f;
    }
};

template <> struct Mfma<FABRIC_FP16> {
    static constexpr int KPL = 8;
    using Frag = f16x8;
    static __device__ inline f32x4 mma(Frag a, Frag b, f32x4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
    static __device__ inline void set(Frag &f, int j, float v) { f[j] = (_Float16)v; }
    static __device__ inline Frag relu(Frag f) { return relu16x8(f); }
    static __device__ inline Frag from8(f32x8 v) { return pack8<Frag, f16x2>(v); }
    static __device__ inline Frag zero()
    {
        Frag f;
        for (int j = 0; j < 8; j++) f[j] = (_Float16)0.0f;
        return f;
    }
};

// ---------------------------------------------------------------------------
// Operand-slot convention of the decoder.  Inside each lane group
// g = lane/16 a lane holds, for its pixel, a list of "slots" c = 0, 1, ...;
// slot c sits in MFMA k-step c / KPL at position c % KPL.  Because the MFMA
// output of lane group g holds neurons 16*mb + 4*g + i, a layer's ReLU output
// becomes the next layer's B operand without moving data between lanes:
// slot c of the next layer carries neuron 16*(c/4) + 4*g + c%4.  The weight
// matrices are permuted to match when they are packed.
//
// Layer inputs per lane group g (slot -> input column, -1 = zero padding):
//   L1: c = 0..3   sin(2 pi frac(2^(k0+c) p_axis))       axis = g/2, k0 = 4*(g%2)
//       c = 4..7   cos(2 pi frac(2^(k0+c-4) p_axis))
//       c = 8, 9   one-blob bins 2g, 2g+1
//   L2, L4: c = 0..15 chained neurons
//   L3: c = 0..15 chained neurons, c = 16, 17 angular inputs:
//       g = 0: (wi.x, wi.y), g = 1: (wi.z, wo.x), g = 2: (wo.y, -), g = 3: (-, -)
// ---------------------------------------------------------------------------
constexpr int kL1Slots = 10;
constexpr int kChainSlots = 16;
constexpr int kL3Slots = 18;

// Column of W1_s (the 40 spatial features, s-index) for L1 slot c of lane group g.
__host__ __device__ inline int l1_feature(int g, int c)
{
    if (c < 8) {
        int axis = g >> 1, k0 = 4 * (g & 1);
        return c < 4 ? 16 * axis + (k0 + c) : 16 * axis + 8 + (k0 + c - 4);
    }
    if (c < 10)
        return 32 + 2 * g + (c - 8);
    return -1;
}

__host__ __device__ inline int chain_neuron(int g, int c)
{
    return 16 * (c >> 2) + 4 * g + (c & 3);
}

// Angular input index (0..4 = wi.x, wi.y, wi.z, wo.x, wo.y) of L3 slot 16 + a.
__host__ __device__ inline int l3_angular(int g, int a)
{
    static const int8_t tab[4][2] = {{0, 1}, {2, 3}, {4, -1}, {-1, -1}};
    return tab[g][a];
}

constexpr int div_up(int a, int b) { return (a + b - 1) / b; }

// Fragment counts per layer for a given K-per-lane.
template <int KPL> struct DecShape {
    static constexpr int KS1 = div_up(kL1Slots, KPL);
    static constexpr int KS2 = div_up(kChainSlots, KPL);
    static constexpr int KS3 = div_up(kL3Slots, KPL);
    static constexpr int KS4 = div_up(kChainSlots, KPL);
    // A fragments: L1-L3 have 4 M-blocks, L4 one (rows 4..15 zero).
    static constexpr int NFRAG = 4 * KS1 + 4 * KS2 + 4 * KS3 + KS4;
    static constexpr int FRAG_L1 = 0;
    static constexpr int FRAG_L2 = FRAG_L1 + 4 * KS1;
    static constexpr int FRAG_L3 = FRAG_L2 + 4 * KS2;
    static constexpr int FRAG_L4 = FRAG_L3 + 4 * KS3;
};

// Packed decoder image for one precision: A fragments [NFRAG][64 lanes][KPL]
// followed by the C-operand biases of L2, L3 (4 M-blocks) and L4 (1 M-block),
// each [64 lanes][4] floats.  L1's bias is per fabric (c_f, with the latent
// folded in) and lives in the context's fabric tables.
constexpr int kBiasFrags = 4 + 4 + 1;

}  // namespace fab
