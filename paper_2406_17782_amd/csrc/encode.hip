// Material encoder forward (Sec. 4.2 "Encoder", in this library's size):
// the weave as a 16x16 one-hot grid plus 12 normalised yarn scalars ->
// e1 = relu(E1 x + c1) -> residual block e2 = relu(e1 + E3 relu(E2 e1 + c2) + c3)
// -> z = E4 e2 + c4.  One 256-thread block per fabric; each dense layer runs
// eight outputs per wavefront at a time with coalesced row reads and a fixed
// butterfly reduction.  It runs once per material edit, not per frame.
#include "enc_dense.hpp"
#include "kernels.hpp"

namespace fab {

namespace {

__global__ __launch_bounds__(256) void encoder_forward_kernel(const float *__restrict__ Q,
                                                              const float *__restrict__ inputs,
                                                              float *__restrict__ latents)
{
    __shared__ float x[kEncIn];
    __shared__ float e1[kEncHid], r2[kEncHid], e2[kEncHid], z[kLatent];
    const int f = blockIdx.x;
    for (int k = threadIdx.x; k < kEncIn; k += blockDim.x)
        x[k] = inputs[(size_t)f * kEncIn + k];
    __syncthreads();
    enc_dense_rows(Q + kOffE1, Q + kOffC1, x, kEncIn, kEncHid, e1, true, nullptr);
    enc_dense_rows(Q + kOffE2, Q + kOffC2, e1, kEncHid, kEncHid, r2, true, nullptr);
    enc_dense_rows(Q + kOffE3, Q + kOffC3, r2, kEncHid, kEncHid, e2, true, e1);
    enc_dense_rows(Q + kOffE4, Q + kOffC4, e2, kEncHid, kLatent, z, false, nullptr);
    for (int k = threadIdx.x; k < kLatent; k += blockDim.x)
        latents[f * kLatent + k] = z[k];
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
    if (n_fabrics <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(encoder_forward_kernel, dim3(n_fabrics), dim3(256), 0, stream, enc_params,
                       enc_inputs, latents);
    return hipGetLastError();
}

}  // namespace fab
