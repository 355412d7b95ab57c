// Layout of the paper-size decoder (Sec. 4.2 "Decoder"): latent 64; the
// footprint's position and size one-blob encoded to 24 channels; layers F1
// F2 (spatial fusion) and A1 .. A5 (angular decoder, A2 and A3 a residual
// block whose input is added before A3's activation); leaky ReLU after every
// layer but A5.  Parameters are row-major W[out][in] followed by b[out],
// layer after layer.
#pragma once

#include "model.hpp"

namespace fab {

constexpr int kPLat = 64;                      // latent size
constexpr int kPBlob = 24;                     // one-blob channels
constexpr int kPX1 = kPLat + kPBlob;           // F1 inputs
constexpr int kPXA1 = 64 + 5;                  // A1 inputs
// Parameter offsets (rows = outputs, row-major), layers F1 F2 A1 A2 A3 A4 A5.
constexpr int kPOffWF1 = 0;
constexpr int kPOffBF1 = kPOffWF1 + 64 * kPX1;
constexpr int kPOffWF2 = kPOffBF1 + 64;
constexpr int kPOffBF2 = kPOffWF2 + 64 * 64;
constexpr int kPOffWA1 = kPOffBF2 + 64;
constexpr int kPOffBA1 = kPOffWA1 + 64 * kPXA1;
constexpr int kPOffWA2 = kPOffBA1 + 64;
constexpr int kPOffBA2 = kPOffWA2 + 64 * 64;
constexpr int kPOffWA3 = kPOffBA2 + 64;
constexpr int kPOffBA3 = kPOffWA3 + 64 * 64;
constexpr int kPOffWA4 = kPOffBA3 + 64;
constexpr int kPOffBA4 = kPOffWA4 + 64 * 64;
constexpr int kPOffWA5 = kPOffBA4 + 64;
constexpr int kPOffBA5 = kPOffWA5 + 4 * 64;
constexpr int kPNDec = kPOffBA5 + 4;
static_assert(kPNDec == FABRIC_N_PAPER_DECODER_PARAMS, "paper decoder layout");
static_assert(kPLat == FABRIC_PAPER_LATENT, "paper latent size");

constexpr float kLeak = 0.01f;

__host__ __device__ inline float lrelu(float x) { return fmaxf(x, kLeak * x); }

// One-blob channels of the footprint (FP32, library functions): circular
// position bins along u and v, then size bins.  raw (the encoding's
// ablation): p_u, p_v and tau in channels 0, 8 and 16, zeros elsewhere.
__device__ inline void blob24(const DevFabric &f, float u, float v, float r, bool raw,
                              float (&x)[24])
{
    const float p[2] = {wrap_period(u, f.fwx, f.inv_wx) * f.inv_wx,
                        wrap_period(v, f.fwy, f.inv_wy) * f.inv_wy};
    if (raw) {
#pragma unroll
        for (int k = 0; k < 24; k++)
            x[k] = 0.0f;
        x[0] = p[0];
        x[8] = p[1];
        x[16] = fminf(fmaxf((log2f(r) + 14.0f) * (1.0f / 16.0f), 0.0f), 1.0f);
        return;
    }
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 8; b++) {
            float d = 8.0f * p[a] - ((float)b + 0.5f);
            d -= 8.0f * floorf((d + 4.0f) * 0.125f);
            x[8 * a + b] = expf(-0.5f * d * d);
        }
    const float tau = fminf(fmaxf((log2f(r) + 14.0f) * (1.0f / 16.0f), 0.0f), 1.0f);
#pragma unroll
    for (int b = 0; b < 8; b++) {
        const float d = 8.0f * tau - ((float)b + 0.5f);
        x[16 + b] = expf(-0.5f * d * d);
    }
}

}  // namespace fab
