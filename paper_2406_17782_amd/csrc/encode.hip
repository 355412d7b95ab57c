// Material encoder forward (Sec. 4.2 "Encoder", in this library's sizes):
// the weave as a 16x16 one-hot grid plus 12 normalised yarn scalars ->
// e1 = relu(E1 x + c1) -> residual block e2 = relu(e1 + E3 relu(E2 e1 + c2) + c3)
// -> z = E4 e2 + c4 (a latent of 32 for the config-size network, 64 for the
// paper-size one).  One 16-wave block per fabric; each dense layer runs
// eight outputs per wavefront at a time with coalesced row reads and a fixed
// butterfly reduction.  It runs once per material edit, not per frame.
#include "enc_dense.hpp"
#include "kernels.hpp"

namespace fab {

namespace {

template <int LAT>
__global__ __launch_bounds__(kEncThreads) void encoder_forward_kernel(const float *__restrict__ Q,
                                                              const float *__restrict__ inputs,
                                                              float *__restrict__ latents)
{
    const int f = blockIdx.x;
    encoder_forward_block<LAT>(Q, inputs + (size_t)f * kEncIn, latents + (size_t)f * LAT);
}

// Latent blends of Sec. 5 "Interpolation" in one block: every thread loads
// its blended values into registers, the block synchronises, then every
// thread stores; so all reads of the table precede all writes and an entry
// may target another entry's source.
constexpr int kLerpThreads = 1024;
constexpr int kLerpPer = FABRIC_MAX_FABRICS * kLatent / kLerpThreads;
static_assert(FABRIC_MAX_FABRICS * kLatent % kLerpThreads == 0, "lerp work split");

__global__ __launch_bounds__(kLerpThreads) void lerp_latents_kernel(
    const LatentLerp *__restrict__ jobs, int count, float *latents)
{
    float val[kLerpPer];
    const int total = count * kLatent;
#pragma unroll
    for (int i = 0; i < kLerpPer; i++) {
        const int e = threadIdx.x + i * kLerpThreads;
        if (e < total) {
            const LatentLerp j = jobs[e / kLatent];
            const int k = e % kLatent;
            const float za = latents[j.a * kLatent + k], zb = latents[j.b * kLatent + k];
            val[i] = fmaf(j.t, zb, (1.0f - j.t) * za);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kLerpPer; i++) {
        const int e = threadIdx.x + i * kLerpThreads;
        if (e < total)
            latents[jobs[e / kLatent].dst * kLatent + e % kLatent] = val[i];
    }
}

}  // namespace

hipError_t launch_lerp_latents(const LatentLerp *jobs, int count, float *latents,
                               hipStream_t stream)
{
    if (count <= 0)
        return hipSuccess;
    if (count > FABRIC_MAX_FABRICS)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(lerp_latents_kernel, dim3(1), dim3(kLerpThreads), 0, stream, jobs, count,
                       latents);
    return hipGetLastError();
}

hipError_t launch_encoder_forward(const float *enc_params, const float *enc_inputs,
                                  int n_fabrics, float *latents, hipStream_t stream)
{
    return launch_encoder_forward_n(enc_params, enc_inputs, n_fabrics, kLatent, latents, stream);
}

hipError_t launch_encoder_forward_n(const float *enc_params, const float *enc_inputs,
                                    int n_fabrics, int lat, float *latents, hipStream_t stream)
{
    if (n_fabrics <= 0)
        return hipSuccess;
    if (lat == kLatent)
        hipLaunchKernelGGL(encoder_forward_kernel<kLatent>, dim3(n_fabrics), dim3(kEncThreads), 0, stream,
                           enc_params, enc_inputs, latents);
    else if (lat == FABRIC_PAPER_LATENT)
        hipLaunchKernelGGL(encoder_forward_kernel<FABRIC_PAPER_LATENT>, dim3(n_fabrics), dim3(kEncThreads),
                           0, stream, enc_params, enc_inputs, latents);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace fab
