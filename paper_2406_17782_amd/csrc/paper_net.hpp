// Layout of the paper-size decoder (Sec. 4.2 "Decoder"): latent 64; the
// footprint's position and size one-blob encoded to 24 channels; layers F1
// F2 (spatial fusion) and A1 .. A5 (angular decoder, A2 and A3 a residual
// block whose input is added before A3's activation); leaky ReLU after every
// layer but A5.  Parameters are row-major W[out][in] followed by b[out],
// layer after layer.
#pragma once

#include "common.hpp"

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

}  // namespace fab
