// Launchers of the library's kernels (host side), implemented in the .hip
// files next to this header and called by fabric_api.cpp.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace fab {

// Pixels a hybrid shading launch routes to the footprint filter.  The
// shading kernel writes one out-of-range bit per pixel (mask[k] covers pixels
// 16k .. 16k+15); launch_queue_build turns the masks into the pixel indices
// idx[0 .. *count) in increasing order (a fixed-order scan, no atomics).
// Sizes: mask ceil(n/32)*2, offsets queue_offset_entries(n), idx n entries.
struct FallbackQueue {
    uint16_t *mask;
    uint32_t *offsets;
    uint32_t *count;
    int32_t *idx;
};

// Footprint filter: one wavefront per pixel at 64 samples and more, one lane
// per pixel below; vis.tex == nullptr for V = 1.
hipError_t launch_gt_filter(const fabric_gbuffer &g, const DevFabric *fabrics, int n_fabrics,
                            int n_samples, uint64_t seed, VisArgs vis, float *out_rgb,
                            float *out_comp, unsigned long long *err, hipStream_t stream);
// The same filter (identical per-pixel results) over the queued pixels of
// a hybrid shading launch, writing their rgb.
hipError_t launch_gt_filter_queue(const fabric_gbuffer &g, const DevFabric *fabrics,
                                  int n_samples, uint64_t seed, VisArgs vis, FallbackQueue q,
                                  float *out_rgb, hipStream_t stream);
size_t queue_offset_entries(int64_t n);
hipError_t launch_queue_build(FallbackQueue q, int64_t n, hipStream_t stream);

// Pack FP32 decoder parameters into the MFMA fragment image of precision prec.
// image must hold decoder_image_bytes(prec).
size_t decoder_image_bytes(int prec);
hipError_t launch_pack_decoder(int prec, const float *dec_params, void *image,
                               hipStream_t stream);

// The image the shading kernel of precision prec reads (32-pixel tiles for
// bf16 / fp16, 16-pixel tiles for fp32).  The bf16 image's neuron scales
// bound the activations over the encoded fabrics' c_f [n_fabrics][64], so it
// is repacked whenever those change.
size_t shade_image_bytes(int prec);
hipError_t launch_pack_shade(int prec, const float *dec_params, const float *cfold, int n_fabrics,
                             void *image, hipStream_t stream);

// FP8-E4M3 shading decoder: calibration over the encoded fabrics, then
// packing with per-layer scales.  image must hold f8_image_bytes().
size_t f8_image_bytes();
hipError_t launch_pack_f8(const float *dec_params, const float *cfold, const DevFabric *fabrics,
                          int n_fabrics, void *image, hipStream_t stream);
hipError_t launch_decode_f8(const fabric_gbuffer &g, const DevFabric *fabrics, int n_fabrics,
                            const float *cfold, const void *image, bool hybrid, FallbackQueue q,
                            float *out, unsigned long long *err, hipStream_t stream);

// c_f = b1 + W1[:, 0:32] z_f for every fabric: cfold[n_fabrics][64].
hipError_t launch_fold_latents(const float *dec_params, const float *latents, int n_fabrics,
                               float *cfold, hipStream_t stream);

// Neural shading.  raw = true writes the decoder's outputs y[4][n] (image from
// launch_pack_decoder); otherwise decoded, albedo-composed rgb[3][n] (image
// from launch_pack_shade).  fallback_samples > 0 routes out-of-range pixels
// to the footprint filter with that many samples (keyed by seed and the
// pixel index as launch_gt_filter): the shading launch marks them in q, the
// queue is compacted in pixel order, and a third launch filters it.
hipError_t launch_decode(int prec, bool raw, const fabric_gbuffer &g, const DevFabric *fabrics,
                         int n_fabrics, const float *cfold, const void *image,
                         int fallback_samples, uint64_t seed, VisArgs vis, FallbackQueue q,
                         float *out, unsigned long long *err, hipStream_t stream);

// One latent blend of Sec. 5 "Interpolation": z[dst] = (1 - t) z[a] + t z[b].
struct LatentLerp {
    int32_t dst, a, b;
    float t;
};
// Apply count (<= FABRIC_MAX_FABRICS) blends, with pairwise distinct dst and
// indices below the table's size, to latents[.][32] in one launch; every
// blend reads the table as it was before the launch.  jobs: device memory.
hipError_t launch_lerp_latents(const LatentLerp *jobs, int count, float *latents,
                               hipStream_t stream);

// The paper-size decoder: image of paper_image_bytes() (the 58 weight
// fragments + the output bias, in BF16 and in FP16), c_f [n_fabrics][64]
// folded from latents [n_fabrics][64]; shading of a G-buffer into rgb [3][n]
// with prec FABRIC_BF16 or FABRIC_FP16 operands.
size_t paper_image_bytes();
// fused = false: the network without the spatial fusion stage (the angular
// inputs enter F1 through A1's angular columns).
hipError_t launch_paper_prepare(const float *params, const float *latents, int n_fabrics,
                                bool fused, void *image, float *cfold, hipStream_t stream);
// raw: footprint inputs without the one-blob encoding (the encoding's ablation).
hipError_t launch_paper_shade(int prec, bool raw, bool fused, const fabric_gbuffer &g,
                              const DevFabric *fabrics, int n_fabrics, const float *cfold,
                              const void *image, float *out, unsigned long long *err,
                              hipStream_t stream);
// FP32 reference of the same network from its FP32 parameters and latents
// (one lane per pixel): rgb [3][n] and/or raw outputs y4 [4][n] (NULL to skip).
hipError_t launch_paper_shade_f32(bool raw, bool fused, const fabric_gbuffer &g,
                                  const DevFabric *fabrics, int n_fabrics, const float *params,
                                  const float *latents, float *out_rgb, float *out_y4,
                                  unsigned long long *err, hipStream_t stream);

// Encoder forward over n_fabrics fabrics: enc_inputs[n][524] -> latents[n][32].
hipError_t launch_encoder_forward(const float *enc_params, const float *enc_inputs,
                                  int n_fabrics, float *latents, hipStream_t stream);
// The same for a latent of `lat` values (32 or FABRIC_PAPER_LATENT; the
// parameters laid out as the config encoder's with E4 [lat][128], c4 [lat]).
hipError_t launch_encoder_forward_n(const float *enc_params, const float *enc_inputs,
                                    int n_fabrics, int lat, float *latents, hipStream_t stream);

}  // namespace fab
