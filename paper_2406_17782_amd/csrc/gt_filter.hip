// Footprint-filtered analytic shading on VALU (Eq. (3)-(5) with V = 1,
// components of Eq. (7), albedo composition of Eq. (8)).  One wavefront owns
// one pixel: its 64 lanes take the pixel's footprint sub-samples (lane,
// lane + 64, ...), accumulate the five sums in FP64 and reduce them with a
// fixed butterfly of wavefront shuffles.
#include "kernels.hpp"
#include "model.hpp"

namespace fab {

namespace {

constexpr int kWavesPerBlock = 4;
constexpr int kXcds = 8;

__global__ __launch_bounds__(256) void gt_filter_kernel(fabric_gbuffer g,
                                                        const DevFabric *__restrict__ fabrics,
                                                        int n_fabrics, int n_samples, int side,
                                                        float inv_side, uint64_t seed,
                                                        float *__restrict__ out_rgb,
                                                        float *__restrict__ out_comp,
                                                        unsigned long long *err)
{
    const int lane = threadIdx.x & 63;
    // Wave-uniform pixel index (keeps the pixel's loads and fabric fields scalar).
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // Workgroups are dealt round-robin to the 8 XCDs; give each XCD one
    // contiguous range of pixels so that an input cache line is fetched into
    // one XCD's L2 only.  gridDim.x is a multiple of kXcds.
    const int per_xcd = gridDim.x / kXcds;
    const int block = (blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
    const int64_t p = (int64_t)block * kWavesPerBlock + wave;
    if (p >= g.n)
        return;
    const int fid = g.fabric_id[p];
    const float u = g.u[p], v = g.v[p], r = g.radius[p];
    const float3 wi = make_float3(g.wi_x[p], g.wi_y[p], g.wi_z[p]);
    const float3 wo = make_float3(g.wo_x[p], g.wo_y[p], g.wo_z[p]);
    const bool fault = pixel_fault(fid, n_fabrics, u, v, r, wi, wo);

    double comp[4] = {0.0, 0.0, 0.0, 0.0};
    if (!fault)
        filter_pixel_wave(fabrics[fid], seed, (uint64_t)p, n_samples, side, inv_side, u, v, r,
                          wi, wo, lane, comp);
    if (lane == 0) {
        const int64_t n = g.n;
        if (fault)
            atomicAdd(err, 1ull);
        if (out_comp) {
            for (int c = 0; c < 4; c++)
                out_comp[c * n + p] = (float)comp[c];
        }
        if (out_rgb) {
            const DevFabric &f = fabrics[fault ? 0 : fid];
            for (int c = 0; c < 3; c++) {
                double rgb = (double)f.kd[0][c] * comp[0] + (double)f.kd[1][c] * comp[1] +
                             (double)f.ks[0][c] * comp[2] + (double)f.ks[1][c] * comp[3];
                out_rgb[c * n + p] = fault ? 0.0f : (float)rgb;
            }
        }
    }
}

}  // namespace

hipError_t launch_gt_filter(const fabric_gbuffer &g, const DevFabric *fabrics, int n_fabrics,
                            int n_samples, uint64_t seed, float *out_rgb, float *out_comp,
                            unsigned long long *err, hipStream_t stream)
{
    if (g.n == 0)
        return hipSuccess;
    int side = 1;
    while (side * side < n_samples)
        side++;
    int64_t blocks = (g.n + kWavesPerBlock - 1) / kWavesPerBlock;
    blocks = (blocks + kXcds - 1) / kXcds * kXcds;   // padding blocks exit at once
    hipLaunchKernelGGL(gt_filter_kernel, dim3((unsigned)blocks), dim3(64 * kWavesPerBlock), 0,
                       stream, g, fabrics, n_fabrics, n_samples, side, 1.0f / (float)side, seed,
                       out_rgb, out_comp, err);
    return hipGetLastError();
}

}  // namespace fab
