// Training of the paper-size decoder (Sec. 4.2 "Decoder", loss of Eq. (9)-(11))
// with one latent of 64 per fabric as a free parameter.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"
#include "train.hpp"

namespace fab {

// Fabrics a paper-size training batch may draw from (the per-fabric latent
// gradient is one split-K job of 64 x n_fabrics entries).
constexpr int kPaperTrainMaxFabrics = 64;

// Device scratch owned by a context, grown on demand.
struct PaperTrainScratch {
    int64_t cap = 0;              // samples the per-sample planes hold
    float *planes = nullptr;      // per-sample planes [801][cap], or in BF16 training
                                  // BF16 planes blocked by 64 samples (see paper_train.hip)
    float *loss_part = nullptr;   // per 256-sample block
    float *loss = nullptr;        // [1]
    float *wt = nullptr;          // transposed weights of F2, A1 (first 64 inputs), A2, A3, A4
    void *bwd_frags = nullptr;    // BF16 transposed-weight fragments of the MFMA backward
    float *partial = nullptr;     // split-K partial weight gradients
    size_t partial_floats = 0;
    float *grad = nullptr;        // [params | latents], or [params | encoder] with the encoder
    float *lat = nullptr;         // [kPaperTrainMaxFabrics][64]: the encoder's latents
    float *enc_acts = nullptr;    // per-fabric encoder backward scratch
    float *dsum = nullptr;        // [fabric][64]: per-fabric sums of F1's input gradient
    int64_t batch_cap = 0;        // generated batch and targets
    uint16_t *b_fid = nullptr;
    float *b_fields = nullptr;    // 9 planes of batch_cap floats
    float *targets = nullptr;     // [4][batch_cap]
};

void paper_train_scratch_free(PaperTrainScratch &s);

// Parameters of the paper-size network's encoder (latent 64).
constexpr int kPaperEncParams = FABRIC_N_PAPER_ENCODER_PARAMS;

struct PaperTrainArgs {
    // [params (FABRIC_N_PAPER_DECODER_PARAMS) | latents [F][64]], or with
    // enc_inputs: [params | encoder parameters (kPaperEncParams)]
    float *master;
    double *adam_m, *adam_v;      // same length
    AdamClock clock;              // the moments' step count
    const DevFabric *fabrics;
    int n_fabrics;
    const fabric_gbuffer *batch;  // NULL: generate
    const float *targets;         // NULL: analytic filter
    fabric_train_cfg cfg;
    unsigned long long *err;
    VisArgs vis;
    bool raw;                     // footprint inputs without the one-blob encoding
    bool fused;                   // false: the angular inputs enter F1 (no spatial fusion)
    const float *enc_inputs;      // NULL: latents are parameters; else the encoder's
                                  // inputs [F][524] and the latents come from the encoder
    // cfg.prec == FABRIC_BF16: the BF16 shading image packed from the
    // current masters and the per-fabric c_f folded from the current latents
    // (the forward's operands); unused for FP32.
    const void *bf16_image;
    const float *cfold;
};

// Parameters Adam updates: the decoder and the latents or the encoder.
inline int64_t paper_trained_count(const PaperTrainArgs &a)
{
    return (int64_t)FABRIC_N_PAPER_DECODER_PARAMS +
           (a.enc_inputs ? (int64_t)kPaperEncParams : (int64_t)a.n_fabrics * FABRIC_PAPER_LATENT);
}

// Loss and gradient [params | latents] (or [params | encoder]) of one batch
// into grad_out (device, paper_trained_count floats).
hipError_t paper_loss_grad(PaperTrainScratch &s, const PaperTrainArgs &a, float *grad_out,
                           float *out_loss, hipStream_t stream);

// One Adam step of the paper-size decoder and its latents (or encoder);
// the latents of the encoder after the step are left in s.lat.  *updated = 0 when
// the loss was non-finite (known only when out_loss != NULL).
hipError_t paper_train_step(PaperTrainScratch &s, const PaperTrainArgs &a, float *out_loss,
                            int *updated, hipStream_t stream);

}  // namespace fab
