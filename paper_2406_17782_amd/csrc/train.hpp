// Training and backward passes of the fabric network (Sec. 4.2, Eq. (9)-(11)).
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace fab {

// Device scratch owned by a context, grown on demand.
struct TrainScratch {
    int64_t cap = 0;            // samples the per-sample buffers hold
    float *acts = nullptr;      // per-sample activations and gradients (see train.hip)
    float *loss_part = nullptr;
    float *partials = nullptr;  // split-K partial weight gradients
    size_t partial_floats = 0;
    float *grad = nullptr;      // [FABRIC_N_PARAMS] full gradient
    float *dcf = nullptr;       // [FABRIC_MAX_FABRICS][64] dL/dc_f
    float *dz = nullptr;        // [FABRIC_MAX_FABRICS][32] dL/dz
    float *enc_acts = nullptr;  // per-fabric encoder activations and their gradients
    float *latents = nullptr;   // [FABRIC_MAX_FABRICS][32]
    float *cfold = nullptr;     // [FABRIC_MAX_FABRICS][64]
    void *fwd_image = nullptr;  // packed forward decoder
    void *bwd_image = nullptr;  // packed transposed decoder
    float *loss = nullptr;      // [1] loss of the last step
    int n_cu = 0;               // compute units of the device (0: not yet queried)
    // generated batch and targets
    int64_t batch_cap = 0;
    uint16_t *b_fid = nullptr;
    float *b_fields = nullptr;  // 9 planes of batch_cap floats
    float *targets = nullptr;   // [4][batch_cap]
};

void train_scratch_free(TrainScratch &s);

// Step count of an Adam state on the device: t [1] (completed updates) and
// the bias corrections of the last counted step, corr [2] = 1 - beta1^t,
// 1 - beta2^t.
struct AdamClock {
    int64_t *t;
    double *corr;
};

struct TrainArgs {
    float *params;
    double *adam_m, *adam_v;
    AdamClock clock;                  // the moments' step count
    const DevFabric *fabrics;
    const float *enc_inputs;
    int n_fabrics;
    const fabric_gbuffer *batch;      // NULL: generate
    const float *targets;             // NULL: analytic filter
    fabric_train_cfg cfg;
    unsigned long long *err;
    VisArgs vis;                      // visibility of generated targets
};

hipError_t launch_make_batch(uint64_t seed, int64_t n, int n_fabrics, float r_lo, float r_hi,
                             float btdf_frac,
                             const fabric_gbuffer_out &out, hipStream_t stream);

// Adam (FP64 moments, FP32 masters) on n parameters; the step is counted
// on the device in clk and skipped, count included, when *loss is not finite.
hipError_t launch_adam(float *params, const float *grad, double *m, double *v, int n,
                       const fabric_train_cfg &cfg, AdamClock clk, const float *loss,
                       hipStream_t stream);

// Decoder backward for explicit parameters and upstream gradients dy[4][n]
// (FP32): grad_params [FABRIC_N_DECODER_PARAMS], grad_latents [F][32].
hipError_t decoder_backward(TrainScratch &s, const fabric_gbuffer &g, const DevFabric *fabrics,
                            int n_fabrics, const float *dec_params, const float *latents,
                            const float *grad_y4, float *grad_params, float *grad_latents,
                            hipStream_t stream);

// Encoder backward: grad_latents [F][32] -> grad_enc_params [FABRIC_N_ENCODER_PARAMS].
hipError_t encoder_backward(TrainScratch &s, const float *enc_params, const float *enc_inputs,
                            int n_fabrics, const float *grad_latents, float *grad_enc_params,
                            hipStream_t stream);

// Loss and full gradient [FABRIC_N_PARAMS] (device grad_out) of one batch.
hipError_t loss_grad(TrainScratch &s, const TrainArgs &a, float *grad_out, float *out_loss,
                     hipStream_t stream);

// One Adam step of encoder + decoder.  *updated = 0 when the loss was
// non-finite (only known when out_loss != NULL; otherwise 1 is reported and
// the device skips the update by itself).
hipError_t train_step(TrainScratch &s, const TrainArgs &a, float *out_loss, int *updated,
                      hipStream_t stream);

}  // namespace fab
