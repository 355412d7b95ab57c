/*
 * fabric.h -- C ABI of the MI355X (gfx950) woven-fabric shading library.
 *
 * The library evaluates, per pixel of a G-buffer, the footprint-filtered
 * reflectance of a woven fabric in two ways:
 *   - neurally: a material latent z (from an encoder of the weave pattern and
 *     yarn parameters) and the pixel's query -- pattern-tiled uv, footprint
 *     radius, light direction wi and view direction wo -- go through a small
 *     decoder MLP that predicts the four components (C_warp, C_weft, S_warp,
 *     S_weft) of Chen, Wang and Wang, "Real-time Neural Woven Fabric
 *     Rendering" (SIGGRAPH 2024), Sec. 4.1 Eq. (7); the reflectance is their
 *     albedo-weighted sum, Eq. (8);
 *   - analytically: the point shading model of Eq. (1)-(2) integrated over the
 *     pixel footprint with the aggregation of Eq. (3)-(5) by stratified
 *     Monte-Carlo samples (visibility V = 1 by default, or the inter-yarn
 *     march of fabric_set_visibility).  This produces the decoder's training
 *     targets (Sec. 4.2, "Loss functions") and serves as its ground truth and
 *     fallback.
 *
 * Conventions shared by every entry point:
 *   - Frames and units.  The macro surface normal is +z.  u runs along +x
 *     (the weft direction), v along +y (the warp direction).  uv and the
 *     footprint radius are in weave cells (one warp x weft crossing = 1).
 *     Directions are unit vectors; wo.z > 0 (the viewer is above the
 *     fabric) and wi.z != 0: wi.z > 0 is reflection, wi.z < 0 light
 *     transmitted from below (Sec. 4.2, the BTDF queries).
 *   - Memory.  Pointers named "device" point to GPU memory of the context's
 *     device; the caller owns them.  "host" pointers are CPU memory.  The
 *     context owns its weights, latents, optimiser state and scratch.
 *   - Streams.  `stream` is a hipStream_t passed as void* (NULL = the null
 *     stream).  Work is enqueued asynchronously on it; only calls that return
 *     host data synchronise.
 *   - Errors.  Every call validates its arguments first and, on failure,
 *     returns a status without enqueuing work.  No C++ exception crosses
 *     the ABI.  Per-pixel input faults (a non-finite field, wi.z == 0,
 *     wo.z <= 0, radius <= 0, fabric_id >= fabrics encoded) do not fail the
 *     call: the pixel's outputs are written as 0 and a device counter is
 *     incremented (read it with fabric_error_count).
 *   - Threading.  A context is not thread-safe; distinct contexts are
 *     independent.
 *   - Determinism.  For fixed inputs and seeds every result is bitwise
 *     repeatable: reductions run in a fixed order.
 */
#ifndef FABRIC_H
#define FABRIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fabric_ctx fabric_ctx;

typedef enum {
    FABRIC_OK = 0,
    FABRIC_E_INVAL = 1,      /* NULL required pointer, bad size or value */
    FABRIC_E_RANGE = 2,      /* a size or count beyond the library's limits */
    FABRIC_E_NOMEM = 3,      /* device allocation failed */
    FABRIC_E_DEVICE = 4,     /* a HIP runtime call failed */
    FABRIC_E_NONFINITE = 5,  /* a training step met a non-finite loss; nothing was updated */
    FABRIC_E_STATE = 6       /* call order: e.g. shading before any fabric was encoded */
} fabric_status;

/* Arithmetic of the decoder's dense layers (all accumulate in FP32). */
typedef enum {
    FABRIC_FP32 = 0,
    FABRIC_BF16 = 1,
    FABRIC_FP16 = 2,
    FABRIC_FP8_E4M3 = 3      /* OCP E4M3 operands with one scale per layer */
} fabric_prec;

#define FABRIC_MAX_FABRICS 256
#define FABRIC_MAX_PERIOD 16
#define FABRIC_LATENT 32
#define FABRIC_N_DECODER_PARAMS 13572
#define FABRIC_N_ENCODER_PARAMS 104352
#define FABRIC_N_PARAMS (FABRIC_N_DECODER_PARAMS + FABRIC_N_ENCODER_PARAMS)
#define FABRIC_MAX_SAMPLES 16384
/* Largest frame of fabric_shade_gbuffer_noalloc (2^22 pixels). */
#define FABRIC_NOALLOC_MAX_PIXELS 4194304
#define FABRIC_PAPER_LATENT 64
#define FABRIC_N_PAPER_DECODER_PARAMS 27076
/* The paper-size network's encoder (E1..E3 as the config encoder's, E4 [64][128], c4 [64]). */
#define FABRIC_N_PAPER_ENCODER_PARAMS 108480

/* One fabric: the weave pattern and the Table 1 parameters per yarn type
 * ([0] = warp, [1] = weft).  Host memory, copied by fabric_encode.
 *   wx, wy       pattern period in cells, 1..16 each
 *   pattern      P[j][i] at pattern[j * wx + i] (first wx*wy bytes):
 *                1 = the warp yarn is on top at column i, row j; 0 = weft
 *   alpha        roughness of the fiber microflake (Eq. (2)), in (0, 1]
 *   beta         height-field scaling, >= 0
 *   twist        twist angle psi (radians), inclination incl = u (radians)
 *   gap          fraction of a cell not covered by the yarn, in [0, 0.9]
 *   wblend       blend weight w of the two Lambertian terms (Eq. (1)), in [0, 1]
 *   kd, ks       RGB diffuse and specular albedos (Eq. (8)); not network
 *                inputs, so editing them needs no re-encode (Sec. 4.3). */
typedef struct {
    uint8_t wx, wy;
    uint8_t pattern[256];
    float alpha[2], beta[2], twist[2], incl[2], gap[2], wblend[2];
    float kd[2][3], ks[2][3];
} fabric_material;

/* A G-buffer of n pixels as device structure-of-arrays, one element per pixel
 * in every array.  fabric_id indexes the fabrics passed to fabric_encode.
 * wi (toward the light) may point below the fabric (wi.z < 0): a
 * transmission query; wo (toward the viewer) points above it.  The library
 * only reads these arrays. */
typedef struct {
    int64_t n;
    const uint16_t *fabric_id;
    const float *u, *v, *radius;
    const float *wi_x, *wi_y, *wi_z, *wo_x, *wo_y, *wo_z;
} fabric_gbuffer;

/* Mutable G-buffer, the output of fabric_make_batch. */
typedef struct {
    int64_t n;
    uint16_t *fabric_id;
    float *u, *v, *radius;
    float *wi_x, *wi_y, *wi_z, *wo_x, *wo_y, *wo_z;
} fabric_gbuffer_out;

/* One training step's settings (fabric_train_step). */
typedef struct {
    int64_t batch;        /* samples drawn when no batch is passed, >= 1 */
    int32_t gt_samples;   /* footprint samples of the analytic targets (perfect square) */
    int32_t prec;         /* fabric_prec of the decoder's forward/backward: FP32 or BF16 */
    uint64_t seed;        /* seed of this step's batch and target samples */
    double lr;            /* Adam learning rate of this step */
    double beta1, beta2, eps;   /* Adam constants, e.g. 0.9, 0.999, 1e-8 */
    float r_lo, r_hi;     /* footprint radius range (cells) of generated batches */
    float btdf_frac;      /* share of generated samples lit from below, in [0, 1] */
} fabric_train_cfg;

/* Create a context on HIP device `device`.  Network parameters are drawn
 * Kaiming-uniform from `seed` (biases 0); Adam moments start at 0.
 * *out receives the context (NULL on failure). */
fabric_status fabric_create(fabric_ctx **out, int device, uint64_t seed);

/* Release every device allocation of the context (waits for its device). */
void fabric_destroy(fabric_ctx *ctx);

/* A static, human-readable name of a status. */
const char *fabric_status_str(fabric_status s);

/* Set the fabric table and run the encoder (Sec. 4.2 "Encoder", Sec. 4.3
 * "Rendering": every material is encoded once before shading).  mats: host
 * array of n_mats (1..FABRIC_MAX_FABRICS) fabrics.  Computes each latent z_f
 * and the decoder's first-layer bias folded with it, c_f = W1_z z_f + b1.
 * Returns E_INVAL on an out-of-range field. */
fabric_status fabric_encode(fabric_ctx *ctx, const fabric_material *mats, int32_t n_mats,
                            void *stream);

/* Albedo edit without re-encoding (Sec. 4.3 "Editing"): replace kd, ks of
 * fabric `fabric` (host arrays [2][3]). */
fabric_status fabric_set_albedo(fabric_ctx *ctx, int32_t fabric, const float kd[2][3],
                                const float ks[2][3], void *stream);

/* Inter-yarn shadowing and masking in the analytic model: the binary
 * visibility V(x_p, w) of Eq. (3) (toward wi, on the integrand) and Eq. (4)
 * (toward wo, on the projected area A and so on the normaliser A_P of
 * Eq. (5)).  enable = 0 (the default): V = 1.  enable = 1: V is the march of
 * a ray over the fabric's height field, whose gradient is the one the ply
 * normals n_p are built from (cross sections and floats integrated from
 * their slopes, lower yarns one cap depth below the top yarns, holes below
 * both), tabulated at 16 x 16 texels per cell in float32; the ray leaves the
 * centre of the point's texel at the texel's height, steps one texel along
 * the major horizontal axis of w per step for up to 32 steps (two cells),
 * and is blocked by a higher texel.  Applies to fabric_gt_filtered, to the
 * fallback pixels of fabric_shade_gbuffer and to targets that
 * fabric_train_step / fabric_loss_grad generate; the decoder is unchanged.
 * The texels are built on the host (FP64, rounded to float32) at the first
 * such call after fabric_encode.  Errors: E_INVAL for enable not 0 or 1. */
fabric_status fabric_set_visibility(fabric_ctx *ctx, int32_t enable);

/* Latent interpolation and extrapolation (Sec. 5 "Interpolation"): the
 * encoder's latents form a space in which a material between two encoded
 * ones is approximated by the weighted blend of their latents, the weight
 * being the position of the varied parameter (e.g. roughness alpha or
 * height-field scale beta) between the two encoded values,
 * t = (p - p_a) / (p_b - p_a); t outside [0, 1] extrapolates.  For
 * k < count:
 *     z[dst[k]] = (1 - t[k]) z[a[k]] + t[k] z[b[k]]
 * computed in FP32 as fma(t, z_b, (1 - t) z_a) (exactly z_a at t = 0 and z_b
 * at t = 1), then c_f = W1_z z_f + b1 refolded.  Every entry reads the latent
 * table as it was before the call, so a dst may also be another entry's a
 * or b.  dst, a, b, t: host arrays of count entries (count in
 * 0..n_mats; 0 does nothing and the arrays may be NULL); indices are fabric
 * slots of the last fabric_encode, the dst values pairwise distinct.  Only
 * latents change: dst keeps its own pattern and albedos from fabric_encode
 * (set them there to the material being approximated).  The next
 * fabric_encode recomputes every latent from the fabric table, replacing
 * edited ones; the FP8 activation scales are recalibrated at the next FP8
 * shading call.  Errors: E_INVAL for a NULL array with count > 0, a
 * repeated dst or a non-finite t; E_RANGE for a count or index out of range;
 * E_STATE before fabric_encode or after a weight change without it.  Returns
 * after the copies of the host arrays; the kernels run on `stream`. */
fabric_status fabric_lerp_latents(fabric_ctx *ctx, const int32_t *dst, const int32_t *a,
                                  const int32_t *b, const float *t, int32_t count, void *stream);

/* The decoder at the paper's own form (Sec. 4.2 "Decoder" and its figure):
 * latent 64; the footprint's position in the pattern period (u, v) and its
 * size one-blob encoded to 24 channels (8 Gaussian bins exp(-d^2/2) each,
 * d in bins; position bins circular, size bins over
 * tau = clamp((log2 r + 14)/16, 0, 1)); spatial fusion by two FC layers
 * over [z, one-blob]; an angular decoder of five FC layers over
 * [spatial feature, wi.xyz, wo.xy], the second and third forming a residual
 * block whose input is added before its last activation; leaky ReLU (0.01)
 * after every layer but the output; width 64.  Outputs decoded and composed
 * as fabric_shade_gbuffer does (k = 100, or 1000 where wi.z < 0).  Shading
 * takes prec FABRIC_BF16 or FABRIC_FP16 operands with FP32 accumulation (the
 * FP16 path applies the leaky ReLU to packed halves) on MFMA, or
 * FABRIC_FP32: the reference, every layer in FP32 from the FP32 parameters
 * and latents (one lane per pixel, not a fast path); training is
 * fabric_paper_train_step.
 *   params   device float [FABRIC_N_PAPER_DECODER_PARAMS], rows = outputs:
 *            WF1[64][88] ([z(64), u bins, v bins, size bins]) bF1[64]
 *            WF2[64][64] bF2 WA1[64][69] ([s(64), wi.xyz, wo.xy]) bA1
 *            WA2[64][64] bA2 WA3[64][64] bA3 WA4[64][64] bA4 WA5[4][64] bA5[4]
 *   latents  device float [n_mats][FABRIC_PAPER_LATENT], for the fabrics of
 *            the last fabric_encode
 * fabric_paper_prepare packs the weights and folds each latent into the
 * first layer (both read on `stream`) and keeps its own copy of both: the
 * masters that fabric_paper_train_step updates (their Adam state is reset
 * here).  fabric_paper_shade then shades
 * like fabric_shade_gbuffer (no fallback), with the fabric table's patterns
 * and albedos.  E_STATE: prepare before any fabric_encode, shade before
 * prepare or after a later fabric_encode. */
fabric_status fabric_paper_prepare(fabric_ctx *ctx, const float *params, const float *latents,
                                   void *stream);
fabric_status fabric_paper_shade(fabric_ctx *ctx, const fabric_gbuffer *g, fabric_prec prec,
                                 float *out_rgb, void *stream);

/* The paper-size network with its latents from an encoder (Sec. 4.2
 * "Encoder", in this library's reading: the residual MLP of
 * fabric_encoder_forward over the same per-fabric inputs, widened to
 * FABRIC_PAPER_LATENT outputs) rather than trained as parameters, so that a
 * fabric never seen in training is shaded from its inputs alone.
 *   params      device float [FABRIC_N_PAPER_DECODER_PARAMS], as
 *               fabric_paper_prepare
 *   enc_params  device float [FABRIC_N_PAPER_ENCODER_PARAMS]: E1[128][524]
 *               c1 E2[128][128] c2 E3[128][128] c3 E4[64][128] c4[64]
 * fabric_paper_prepare_encoder keeps its own copy of both (the masters that
 * fabric_paper_train_step then updates together, Adam state reset), encodes
 * the current fabric table and packs the shading image, all on `stream`.
 * fabric_paper_encode re-encodes the table of the last fabric_encode with
 * the current masters (a new table of unseen fabrics, for instance) and
 * re-packs; fabric_paper_prepare leaves encoder mode.  In encoder mode
 * fabric_paper_get_params returns the encoder's latents, and
 * fabric_paper_get_encoder copies enc_params to host (synchronises).
 * Errors: E_INVAL for NULL pointers; E_STATE before any fabric_encode, and
 * for encode and get_encoder outside encoder mode. */
fabric_status fabric_paper_prepare_encoder(fabric_ctx *ctx, const float *params,
                                           const float *enc_params, void *stream);
fabric_status fabric_paper_encode(fabric_ctx *ctx, void *stream);
fabric_status fabric_paper_get_encoder(fabric_ctx *ctx, float *enc_params_host);

/* The paper-size decoder's raw outputs (y of Sec. 4.2 before the decoding of
 * Eq. (9): C_warp, C_weft, S_warp, S_weft in the log-mapped domain), in FP32
 * from the parameters and latents of the last fabric_paper_prepare or
 * fabric_paper_train_step, as fabric_paper_shade's FP32 reference computes
 * them.  y4: device float [4][n]; faulted pixels give 0 and are counted.
 * Errors as fabric_paper_shade. */
fabric_status fabric_paper_forward(fabric_ctx *ctx, const fabric_gbuffer *g, float *y4,
                                   void *stream);

/* Neural shading of a G-buffer (Sec. 4.3 "Rendering"): per pixel, the
 * decoder's four outputs decoded as C = max(y, 0), S = max((e^y - 1)/k, 0)
 * with k = 100, or 1000 where wi.z < 0 (transmission, Sec. 4.2)
 * (inverse of the specular mapping of Eq. (9)) and composed with Eq. (8).
 *   prec              arithmetic of the dense layers: FP32; BF16 or FP16
 *                     operands with FP32 accumulation; FP8_E4M3 operands with
 *                     FP32 accumulation and one power-of-two scale per layer
 *                     for the weights and one for the activations.  The FP8
 *                     activation scales are calibrated on the device (the
 *                     largest hidden activations over a fixed synthetic batch
 *                     drawn from the encoded fabrics) at the first FP8 call
 *                     after fabric_encode or a parameter change, so they never
 *                     depend on the frame being shaded; activations above the
 *                     calibrated range saturate at the largest E4M3 value.
 *   fallback_samples  0: every pixel is shaded by the decoder.  > 0 (a perfect
 *                     square <= FABRIC_MAX_SAMPLES): pixels outside the
 *                     network's range (radius > 1 cell or wo.z < 0.05) are
 *                     instead shaded, in the same call and on the same
 *                     stream, by the analytic footprint filter with that many
 *                     samples, keyed by `seed` and the pixel index exactly as
 *                     fabric_gt_filtered (bitwise the same values).  The
 *                     shading launch marks them; a fixed-order compaction
 *                     queues them in pixel order for the filter launch.
 *   out_rgb           device float [3][n] (R plane, G plane, B plane).
 * Requires fabric_encode after the last weight change (else E_STATE). */
fabric_status fabric_shade_gbuffer(fabric_ctx *ctx, const fabric_gbuffer *g, fabric_prec prec,
                                   int32_t fallback_samples, uint64_t seed, float *out_rgb,
                                   void *stream);

/* fabric_shade_gbuffer for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, same kernels and bitwise the same results as
 * fabric_shade_gbuffer, but the hybrid fallback queue (out-of-range mask,
 * scan offsets, count, pixel indices) lives in a fixed device array of the
 * library (20 MiB per GPU, held until the process ends) instead of context
 * memory, and the call allocates nothing.  Nothing in the array needs to
 * start at zero: each call rewrites the parts it reads.  Every call on one
 * GPU shares that GPU's array, so calls that overlap on one GPU (any
 * contexts, any streams) race and must be serialised by the caller.
 * Errors: as fabric_shade_gbuffer; E_RANGE when n exceeds
 * FABRIC_NOALLOC_MAX_PIXELS; E_STATE when visibility is on with fallback
 * and the height texels of the current fabric table have not been built yet
 * (any call of fabric_gt_filtered or fabric_shade_gbuffer with fallback
 * builds them). */
fabric_status fabric_shade_gbuffer_noalloc(fabric_ctx *ctx, const fabric_gbuffer *g,
                                           fabric_prec prec, int32_t fallback_samples,
                                           uint64_t seed, float *out_rgb, void *stream);

/* Footprint-filtered analytic shading (Eq. (3)-(5), with V as set by
 * fabric_set_visibility; components of Eq. (7)).  Pixel p's footprint is the disk of radius radius[p] about
 * (u[p], v[p]) with a uniform kernel; n_samples = m*m stratified samples,
 * stratum k = ky*m + kx jittered by the (p*n_samples + k)-th output of
 * SplitMix64 seeded with `seed` (upper 24 bits for x, bits 39..16 for y) and
 * mapped to the disk with the Shirley-Chiu concentric map.  Per sample:
 * rho = f * <wi.n_p> and projected area <wo.n_p>/<n_s.n_p> (holes: wo.z).
 * Light below the fabric (wi.z < 0) is transmitted by plies it reaches from
 * below: f_s is the single scattering of the specular slab between its
 * faces, D / (4 |ci| co) (e^{-2 Lambda_o} - e^{-2 Lambda_i}) /
 * (Lambda_i - Lambda_o), f_d the Lambertian share (1 - w)/pi, the cosine
 * |wi.n_p|; holes transmit nothing (no delta transmission);
 * C_y = sum[yarn = y] rho_d A / sum A, S_y likewise, summed in FP64.
 *   out_comp  device float [4][n] (C_warp, C_weft, S_warp, S_weft) or NULL
 *   out_rgb   device float [3][n] (Eq. (8)) or NULL (not both NULL). */
fabric_status fabric_gt_filtered(fabric_ctx *ctx, const fabric_gbuffer *g, int32_t n_samples,
                                 uint64_t seed, float *out_rgb, float *out_comp, void *stream);

/* Decoder forward with explicit parameters (for autograd wrappers).
 *   dec_params  device float [FABRIC_N_DECODER_PARAMS]: W1[64][72] b1[64]
 *               W2[64][64] b2[64] W3[64][69] b3[64] W4[4][64] b4[4], rows =
 *               output units; W1's columns are [z(32), s(40)], W3's
 *               [h2(64), wi.x, wi.y, wi.z, wo.x, wo.y]
 *   latents     device float [n_mats][32]
 *   y4          device float [4][n]: raw outputs (C_warp, C_weft, S_warp, S_weft
 *               in the log-mapped domain of Eq. (9)).
 * prec is FABRIC_FP32 or FABRIC_BF16.  Uses the fabric table of the last
 * fabric_encode for the pattern periods. */
fabric_status fabric_decoder_forward(fabric_ctx *ctx, const fabric_gbuffer *g, fabric_prec prec,
                                     const float *dec_params, const float *latents, float *y4,
                                     void *stream);

/* Decoder backward: given dL/dy4 (device [4][n]), write dL/d(dec_params)
 * (device float [FABRIC_N_DECODER_PARAMS], overwritten) and dL/dlatents
 * (device float [n_mats][32], overwritten).  FP32 arithmetic; the sums over
 * pixels are reduced in a fixed order. */
fabric_status fabric_decoder_backward(fabric_ctx *ctx, const fabric_gbuffer *g,
                                      const float *dec_params, const float *latents,
                                      const float *grad_y4, float *grad_params,
                                      float *grad_latents, void *stream);

/* Encoder forward with explicit parameters over the encoded fabric table:
 * enc_params device float [FABRIC_N_ENCODER_PARAMS]; latents device [n_mats][32]. */
fabric_status fabric_encoder_forward(fabric_ctx *ctx, const float *enc_params, float *latents,
                                     void *stream);

/* Encoder backward: dL/dlatents (device [n_mats][32]) -> dL/d(enc_params)
 * (device float [FABRIC_N_ENCODER_PARAMS], overwritten). */
fabric_status fabric_encoder_backward(fabric_ctx *ctx, const float *enc_params,
                                      const float *grad_latents, float *grad_enc_params,
                                      void *stream);

/* Draw a training batch: sample q takes the outputs 8q..8q+5 of SplitMix64
 * seeded with `seed`: fabric id = (z >> 32) mod n_mats; (u, v) = 8 * two
 * 24-bit uniforms; radius log-uniform on [r_lo, r_hi]; wi and wo
 * cosine-weighted from two 24-bit uniforms each; wi is turned below the
 * fabric (wi.z negated: a transmission query, Sec. 4.2) when the upper 24
 * bits of output 8q+5, as a uniform in [0, 1), are below btdf_frac.  out
 * arrays: device, n each.  E_INVAL for btdf_frac outside [0, 1]. */
fabric_status fabric_make_batch(fabric_ctx *ctx, uint64_t seed, int64_t n, float r_lo,
                                float r_hi, float btdf_frac, const fabric_gbuffer_out *out,
                                void *stream);

/* One optimisation step of encoder + decoder on the encoded fabric table:
 * loss of Eq. (9)-(11) (lambda_S = 0.4, lambda_C = 0.1, k = 100 for samples
 * lit from above and 1000 for samples lit from below), gradients
 * by hand-written backward kernels, Adam with FP64 moments on FP32 masters.
 * The loss is summed in FP32 in a fixed order with compensated (Kahan)
 * sums; Adam's step count lives on the device with its moments, so a step
 * skipped for a non-finite loss is not counted, out_loss given or not.
 *   batch        device G-buffer, or NULL to draw cfg->batch samples with
 *                fabric_make_batch(cfg->seed)
 *   targets      device float [4][n] components (only with a batch), or NULL
 *                to compute them with the analytic filter (cfg->gt_samples
 *                samples, seed cfg->seed ^ 1)
 *   out_loss     host float, or NULL for no synchronisation
 * A non-finite loss leaves weights, moments and step count unchanged and
 * returns E_NONFINITE (reported only when out_loss is given).  After a step,
 * shading needs fabric_encode again (E_STATE otherwise). */
fabric_status fabric_train_step(fabric_ctx *ctx, const fabric_gbuffer *batch,
                                const float *targets, const fabric_train_cfg *cfg,
                                float *out_loss, void *stream);

/* Loss of Eq. (9)-(11) and its gradient with respect to all parameters,
 * without an update: the first half of fabric_train_step (same arguments and
 * batch/target rules).  grad: device float [FABRIC_N_PARAMS] (overwritten),
 * laid out like fabric_get_params.  out_loss: host float or NULL. */
fabric_status fabric_loss_grad(fabric_ctx *ctx, const fabric_gbuffer *batch, const float *targets,
                               const fabric_train_cfg *cfg, float *grad, float *out_loss,
                               void *stream);

/* Training of the paper-size decoder (Sec. 4.2 "Decoder", loss of
 * Eq. (9)-(11)) on the context's masters from fabric_paper_prepare, with
 * one latent of FABRIC_PAPER_LATENT per fabric trained as a parameter, or
 * from fabric_paper_prepare_encoder, with the encoder trained beside the
 * decoder (the paper's convolutional encoder of normal and orientation maps
 * is not part of this library).  The batch, targets and cfg behave as for fabric_train_step
 * (generated batch and 256-sample targets by default, visibility as set by
 * fabric_set_visibility).  cfg->prec is FABRIC_FP32 (forward and backward
 * in FP32 on the vector units, one sample per lane) or FABRIC_BF16 (forward
 * and backward on the matrix cores, 32 samples per wave: BF16 operands,
 * the forward's from the shading image of the current masters, the
 * backward's from the transposed masters, FP32 accumulation, per-sample
 * activations and gradients kept as BF16); the weight gradients are
 * fixed-order split-K sums over the per-sample values (FP32 or BF16
 * operands, FP32 sums), the masters stay FP32 and Adam keeps FP64 moments,
 * so repeated runs are bitwise equal.  Other precisions: E_INVAL.
 * fabric_paper_train_step takes one Adam step over [params | latents]
 * ([params | enc_params] in encoder mode) and re-packs the shading image
 * from the updated masters; a non-finite loss (known only when
 * out_loss != NULL) skips the update and returns E_NONFINITE.
 * fabric_paper_loss_grad writes the gradient to device `grad`
 * [FABRIC_N_PAPER_DECODER_PARAMS + n_mats * FABRIC_PAPER_LATENT]
 * (parameter layout of fabric_paper_prepare, then the latents), in encoder
 * mode [FABRIC_N_PAPER_DECODER_PARAMS + FABRIC_N_PAPER_ENCODER_PARAMS].
 * Errors: as fabric_train_step; E_STATE before fabric_paper_prepare or
 * after a later fabric_encode (until fabric_paper_encode in encoder mode);
 * E_RANGE for more than 64 fabrics. */
fabric_status fabric_paper_train_step(fabric_ctx *ctx, const fabric_gbuffer *batch,
                                      const float *targets, const fabric_train_cfg *cfg,
                                      float *out_loss, void *stream);
fabric_status fabric_paper_loss_grad(fabric_ctx *ctx, const fabric_gbuffer *batch,
                                     const float *targets, const fabric_train_cfg *cfg, float *grad,
                                     float *out_loss, void *stream);
/* Footprint encoding of the paper-size decoder's shading and training:
 * one_blob = 1 (the default) is the one-blob encoding of Sec. 4.2; 0 feeds
 * the unencoded inputs instead (the ablation of Sec. 5 "Encoding of
 * footprint"): the position fractions (u mod W_x)/W_x, (v mod W_y)/W_y and
 * tau = clamp((log2 r + 14)/16, 0, 1) in the first channel of their bins,
 * the other channels 0; the parameter layout is unchanged.  A network is
 * shaded with the encoding it was trained with.  E_INVAL unless 0 or 1. */
fabric_status fabric_paper_set_footprint_encoding(fabric_ctx *ctx, int32_t one_blob);
/* Wiring of the paper-size decoder's shading and training: fused = 1 (the
 * default) is the paper's network, the angular inputs entering A1 after the
 * spatial fusion F1, F2; fused = 0 removes the fusion stage (the ablation of
 * Sec. 5 "Spatial fusion"): wi.xyz and wo.xy enter F1 beside the latent and
 * the footprint, weighted by A1's angular columns, and A1 sees zeros in
 * their place, so all seven layers follow the concatenated input and the
 * parameter layout is unchanged.  Re-packs the shading image of the prepared
 * masters on `stream`.  A network is shaded with the wiring it was trained
 * with.  E_INVAL unless 0 or 1. */
fabric_status fabric_paper_set_spatial_fusion(fabric_ctx *ctx, int32_t fused, void *stream);
/* The paper-size masters to host: params [FABRIC_N_PAPER_DECODER_PARAMS],
 * latents [n_mats][FABRIC_PAPER_LATENT].  Synchronises the device.  E_STATE
 * before fabric_paper_prepare. */
fabric_status fabric_paper_get_params(fabric_ctx *ctx, float *params_host, float *latents_host);

/* Parameters as one FP32 vector [FABRIC_N_PARAMS] = [decoder | encoder]
 * (layouts as in fabric_decoder_forward and fabric_encoder_forward; encoder:
 * E1[128][524] c1 E2[128][128] c2 E3[128][128] c3 E4[32][128] c4).  host
 * memory; both synchronise.  set resets nothing else (Adam state persists). */
fabric_status fabric_get_params(fabric_ctx *ctx, float *host, size_t count);
fabric_status fabric_set_params(fabric_ctx *ctx, const float *host, size_t count);

/* Latents of the encoded fabrics, host float [n_mats][32] (synchronises). */
fabric_status fabric_get_latents(fabric_ctx *ctx, float *host, int32_t n_mats);

/* Checkpoint: parameters, Adam moments and step as one little-endian blob
 * (magic "FABRICK1", version, counts).  With host == NULL, *bytes receives the
 * size needed; otherwise *bytes must hold at least that.  Both synchronise. */
fabric_status fabric_save(fabric_ctx *ctx, void *host, size_t *bytes);
fabric_status fabric_load(fabric_ctx *ctx, const void *host, size_t bytes);

/* Number of pixel faults counted since the last reset (synchronises);
 * reset != 0 clears the counter. */
int64_t fabric_error_count(fabric_ctx *ctx, int reset);

#ifdef __cplusplus
}
#endif

#endif /* FABRIC_H */
