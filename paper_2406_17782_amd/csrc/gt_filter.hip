// Footprint-filtered analytic shading on VALU (Eq. (3)-(5), with V = 1 or
// the inter-yarn visibility march of the height field, components of
// Eq. (7), albedo composition of Eq. (8)).  At 64 samples and more one
// wavefront owns one pixel: its 64 lanes take the pixel's footprint
// sub-samples (lane, lane + 64, ...), accumulate the five sums in FP64 and
// reduce them with a fixed butterfly of wavefront shuffles.  Below 64
// samples each lane owns one pixel and takes its samples in order.
#include "kernels.hpp"
#include "model.hpp"
#include "shade.hpp"

namespace fab {

namespace {

// One lane's FP64 footprint estimate for its own pixel: samples k = 0 ..
// N - 1 in order (the same sample positions as the wave-wide estimate, the
// five sums added in sample order).  For footprints of fewer than 64
// samples, where a wave per pixel would leave lanes idle.
template <bool VIS, bool POW2>
__device__ inline void filter_pixel_lane(const DevFabric &f, uint64_t seed, uint64_t pixel,
                                         int n_samples, int side, float u,
                                         float v, float r, float3 wi, float3 wo,
                                         const float *tex, const VisFabric &vf, double comp[4])
{
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    uint64_t state = seed + ((uint64_t)pixel * (uint64_t)n_samples + 1ull) * kGoldenGamma;
    int kx = 0, ky = 0;
    for (int k = 0; k < n_samples; k++, state += kGoldenGamma) {
        float2 pos = footprint_sample<POW2>(splitmix64_mix(state), kx, ky, (float)side, u, v, r);
        if (++kx == side) {
            kx = 0;
            ky += 1;
        }
        SampleVal sv = eval_surface_point<VIS>(f, pos.x, pos.y, wi, wo, tex, vf);
        double nc = sv.num_c, ns = sv.num_s;
        acc[0] += sv.yarn == kWarp ? nc : 0.0;
        acc[1] += sv.yarn == kWeft ? nc : 0.0;
        acc[2] += sv.yarn == kWarp ? ns : 0.0;
        acc[3] += sv.yarn == kWeft ? ns : 0.0;
        acc[4] += (double)sv.area;
    }
    for (int c = 0; c < 4; c++)
        comp[c] = acc[4] > 0.0 ? acc[c] / acc[4] : 0.0;
}

constexpr int kWavesPerBlock = 4;
constexpr int kXcds = 8;

// Pixel p by the wave (LANE = false; lane 0 writes) or by one lane (LANE =
// true): the filter's components and Eq. (8) composition (faulty inputs:
// zeros and one count).
template <bool VIS, bool LANE>
__device__ inline void filter_one_pixel(const fabric_gbuffer &g, const DevFabric *__restrict__ fabrics,
                                        int n_fabrics, int64_t p, int n_samples, int side,
                                        uint64_t seed, int lane, VisArgs vis,
                                        float *__restrict__ out_rgb, float *__restrict__ out_comp,
                                        unsigned long long *err)
{
    const int fid = g.fabric_id[p];
    const float u = g.u[p], v = g.v[p], r = g.radius[p];
    const float3 wi = make_float3(g.wi_x[p], g.wi_y[p], g.wi_z[p]);
    const float3 wo = make_float3(g.wo_x[p], g.wo_y[p], g.wo_z[p]);
    const bool fault = pixel_fault(fid, n_fabrics, u, v, r, wi, wo);

    double comp[4] = {0.0, 0.0, 0.0, 0.0};
    if (!fault) {
        const VisFabric vf = VIS ? vis.fab[fid] : VisFabric{0, 0, 0, 0.0f};
        // side is the same for every pixel of the launch: a uniform branch.
        const bool pow2 = is_pow2(side);
        if (LANE && pow2)
            filter_pixel_lane<VIS, true>(fabrics[fid], seed, (uint64_t)p, n_samples, side, u,
                                         v, r, wi, wo, vis.tex, vf, comp);
        else if (LANE)
            filter_pixel_lane<VIS, false>(fabrics[fid], seed, (uint64_t)p, n_samples, side, u,
                                          v, r, wi, wo, vis.tex, vf, comp);
        else if (pow2)
            filter_pixel_wave<VIS, true>(fabrics[fid], seed, (uint64_t)p, n_samples, side, u,
                                         v, r, wi, wo, lane, vis.tex, vf, comp);
        else
            filter_pixel_wave<VIS, false>(fabrics[fid], seed, (uint64_t)p, n_samples, side, u,
                                          v, r, wi, wo, lane, vis.tex, vf, comp);
    }
    if (LANE || lane == 0) {
        const int64_t n = g.n;
        if (fault && err)
            atomicAdd(err, 1ull);
        if (out_comp) {
            for (int c = 0; c < 4; c++)
                out_comp[c * n + p] = (float)comp[c];
        }
        if (out_rgb) {
            const DevFabric &f = fabrics[fault ? 0 : fid];
            const float c0 = (float)comp[0], c1 = (float)comp[1], c2 = (float)comp[2],
                        c3 = (float)comp[3];
            for (int c = 0; c < 3; c++) {
                const float rgb = f.kd[0][c] * c0 + f.kd[1][c] * c1 + f.ks[0][c] * c2 +
                                  f.ks[1][c] * c3;
                out_rgb[c * n + p] = fault ? 0.0f : rgb;
            }
        }
    }
}

template <bool VIS>
__global__ __launch_bounds__(256) void gt_filter_kernel(fabric_gbuffer g,
                                                        const DevFabric *__restrict__ fabrics,
                                                        int n_fabrics, int n_samples, int side,
                                                        uint64_t seed, VisArgs vis,
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
    filter_one_pixel<VIS, false>(g, fabrics, n_fabrics, p, n_samples, side, seed, lane,
                                 vis, out_rgb, out_comp, err);
}

// Fewer than 64 samples: one lane per pixel, 256 consecutive pixels per
// workgroup, with the same XCD-contiguous block order as above.
template <bool VIS>
__global__ __launch_bounds__(256) void gt_filter_lane_kernel(fabric_gbuffer g,
                                                             const DevFabric *__restrict__ fabrics,
                                                             int n_fabrics, int n_samples, int side,
                                                             uint64_t seed,
                                                             VisArgs vis, float *__restrict__ out_rgb,
                                                             float *__restrict__ out_comp,
                                                             unsigned long long *err)
{
    const int per_xcd = gridDim.x / kXcds;
    const int block = (blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
    const int64_t p = (int64_t)block * blockDim.x + threadIdx.x;
    if (p >= g.n)
        return;
    filter_one_pixel<VIS, true>(g, fabrics, n_fabrics, p, n_samples, side, seed, 0, vis,
                                out_rgb, out_comp, err);
}

// The queued pixels of a hybrid shading launch (all valid and in range of
// the fabric table), in increasing pixel order: one wave per queue slot,
// like gt_filter_kernel; the grid covers every pixel of the frame and the
// waves past the queue's length exit at once (the length is only known on
// the device).
template <bool VIS>
__global__ __launch_bounds__(256) void gt_filter_queue_kernel(fabric_gbuffer g,
                                                              const DevFabric *__restrict__ fabrics,
                                                              int n_samples, int side,
                                                              uint64_t seed,
                                                              VisArgs vis, FallbackQueue q,
                                                              float *__restrict__ out_rgb)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t k = blockIdx.x * kWavesPerBlock + wave;
    if (k >= *q.count)
        return;
    const int64_t p = __builtin_amdgcn_readfirstlane(q.idx[k]);
    filter_one_pixel<VIS, false>(g, fabrics, FABRIC_MAX_FABRICS, p, n_samples, side,
                                 seed, lane, vis, out_rgb, nullptr, nullptr);
}

// The queue below 64 samples: one lane per queue slot, each pixel computed
// exactly as gt_filter_lane_kernel computes it.
template <bool VIS>
__global__ __launch_bounds__(256) void gt_filter_queue_lane_kernel(fabric_gbuffer g,
                                                                   const DevFabric *__restrict__ fabrics,
                                                                   int n_samples, int side,
                                                                   uint64_t seed,
                                                                   VisArgs vis, FallbackQueue q,
                                                                   float *__restrict__ out_rgb)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)*q.count)
        return;
    filter_one_pixel<VIS, true>(g, fabrics, FABRIC_MAX_FABRICS, (int64_t)q.idx[k], n_samples, side,
                                seed, 0, vis, out_rgb, nullptr, nullptr);
}

constexpr int kLaneBelow = 64;   // sample counts below this take one lane per pixel

// Queue compaction in three fixed-order steps (no atomics).  The offsets
// buffer holds the per-group local offsets [ngroups], then the per-block
// totals [nblk] and the blocks' exclusive prefixes [nblk].
constexpr int kScanGroupsPerThread = 8;
constexpr int kScanBlock = 256;
constexpr int kScanGroupsPerBlock = kScanBlock * kScanGroupsPerThread;   // 2048 groups

// Step 1: per block, offsets of its groups relative to the block, and the
// block's total.  Thread t takes 8 consecutive groups (one 16-byte load).
__global__ __launch_bounds__(kScanBlock) void queue_scan_local_kernel(
    const uint16_t *__restrict__ mask, int64_t ngroups, uint32_t *__restrict__ offsets,
    uint32_t *__restrict__ block_sums)
{
    __shared__ uint32_t part[kScanBlock];
    const int t = threadIdx.x;
    const int64_t k0 = (int64_t)blockIdx.x * kScanGroupsPerBlock + t * kScanGroupsPerThread;
    uint32_t c[kScanGroupsPerThread];
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < kScanGroupsPerThread; j++) {
        c[j] = k0 + j < ngroups ? (uint32_t)__popc((uint32_t)mask[k0 + j]) : 0u;
        sum += c[j];
    }
    part[t] = sum;
    __syncthreads();
    for (int d = 1; d < kScanBlock; d <<= 1) {   // inclusive scan of the thread sums
        const uint32_t add = t >= d ? part[t - d] : 0u;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    uint32_t run = part[t] - sum;
#pragma unroll
    for (int j = 0; j < kScanGroupsPerThread; j++) {
        if (k0 + j < ngroups)
            offsets[k0 + j] = run;
        run += c[j];
    }
    if (t == kScanBlock - 1)
        block_sums[blockIdx.x] = part[t];
}

// Step 2 (one block): exclusive prefixes of the block totals, and the count.
__global__ __launch_bounds__(1024) void queue_scan_blocks_kernel(const uint32_t *__restrict__ block_sums,
                                                                int nblk,
                                                                uint32_t *__restrict__ block_prefix,
                                                                uint32_t *__restrict__ count)
{
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int per = (nblk + 1023) / 1024;
    const int b0 = t * per, b1 = b0 + per < nblk ? b0 + per : nblk;
    uint32_t sum = 0;
    for (int b = b0; b < b1; b++)
        sum += block_sums[b];
    part[t] = sum;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const uint32_t add = t >= d ? part[t - d] : 0u;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    uint32_t run = part[t] - sum;
    for (int b = b0; b < b1; b++) {
        block_prefix[b] = run;
        run += block_sums[b];
    }
    if (t == 1023)
        *count = part[t];
}

// Step 3: each 16-pixel group writes its marked pixels' indices, in
// increasing order, from its offset.
__global__ void queue_scatter_kernel(const uint16_t *__restrict__ mask,
                                     const uint32_t *__restrict__ offsets,
                                     const uint32_t *__restrict__ block_prefix, int64_t ngroups,
                                     int32_t *__restrict__ idx)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ngroups)
        return;
    uint32_t bits = mask[k];
    uint32_t o = offsets[k] + block_prefix[k / kScanGroupsPerBlock];
    while (bits) {
        const int b = __builtin_ctz(bits);
        bits &= bits - 1u;
        idx[o++] = (int32_t)(16 * k + b);
    }
}

}  // namespace

hipError_t launch_gt_filter(const fabric_gbuffer &g, const DevFabric *fabrics, int n_fabrics,
                            int n_samples, uint64_t seed, VisArgs vis, float *out_rgb,
                            float *out_comp, unsigned long long *err, hipStream_t stream)
{
    if (g.n == 0)
        return hipSuccess;
    const int side = sample_side(n_samples);
    if (n_samples < kLaneBelow) {
        int64_t blocks = (g.n + 255) / 256;
        blocks = (blocks + kXcds - 1) / kXcds * kXcds;   // padding blocks exit at once
        if (vis.tex)
            hipLaunchKernelGGL(gt_filter_lane_kernel<true>, dim3((unsigned)blocks), dim3(256), 0,
                               stream, g, fabrics, n_fabrics, n_samples, side,
                               seed, vis, out_rgb, out_comp, err);
        else
            hipLaunchKernelGGL(gt_filter_lane_kernel<false>, dim3((unsigned)blocks), dim3(256), 0,
                               stream, g, fabrics, n_fabrics, n_samples, side,
                               seed, vis, out_rgb, out_comp, err);
        return hipGetLastError();
    }
    int64_t blocks = (g.n + kWavesPerBlock - 1) / kWavesPerBlock;
    blocks = (blocks + kXcds - 1) / kXcds * kXcds;   // padding blocks exit at once
    if (vis.tex)
        hipLaunchKernelGGL(gt_filter_kernel<true>, dim3((unsigned)blocks), dim3(64 * kWavesPerBlock),
                           0, stream, g, fabrics, n_fabrics, n_samples, side,
                           seed, vis, out_rgb, out_comp, err);
    else
        hipLaunchKernelGGL(gt_filter_kernel<false>, dim3((unsigned)blocks), dim3(64 * kWavesPerBlock),
                           0, stream, g, fabrics, n_fabrics, n_samples, side,
                           seed, vis, out_rgb, out_comp, err);
    return hipGetLastError();
}

hipError_t launch_gt_filter_queue(const fabric_gbuffer &g, const DevFabric *fabrics,
                                  int n_samples, uint64_t seed, VisArgs vis, FallbackQueue q,
                                  float *out_rgb, hipStream_t stream)
{
    if (g.n == 0)
        return hipSuccess;
    const int side = sample_side(n_samples);
    if (n_samples < kLaneBelow) {
        const int64_t blocks = (g.n + 255) / 256;
        if (vis.tex)
            hipLaunchKernelGGL(gt_filter_queue_lane_kernel<true>, dim3((unsigned)blocks), dim3(256),
                               0, stream, g, fabrics, n_samples, side, seed,
                               vis, q, out_rgb);
        else
            hipLaunchKernelGGL(gt_filter_queue_lane_kernel<false>, dim3((unsigned)blocks), dim3(256),
                               0, stream, g, fabrics, n_samples, side, seed,
                               vis, q, out_rgb);
        return hipGetLastError();
    }
    const int64_t blocks = (g.n + kWavesPerBlock - 1) / kWavesPerBlock;
    if (vis.tex)
        hipLaunchKernelGGL(gt_filter_queue_kernel<true>, dim3((unsigned)blocks),
                           dim3(64 * kWavesPerBlock), 0, stream, g, fabrics, n_samples, side,
                           seed, vis, q, out_rgb);
    else
        hipLaunchKernelGGL(gt_filter_queue_kernel<false>, dim3((unsigned)blocks),
                           dim3(64 * kWavesPerBlock), 0, stream, g, fabrics, n_samples, side,
                           seed, vis, q, out_rgb);
    return hipGetLastError();
}

size_t queue_offset_entries(int64_t n)
{
    const int64_t ngroups = (n + 15) / 16;
    const int64_t nblk = (ngroups + kScanGroupsPerBlock - 1) / kScanGroupsPerBlock;
    return (size_t)(ngroups + 2 * nblk);
}

hipError_t launch_queue_build(FallbackQueue q, int64_t n, hipStream_t stream)
{
    const int64_t ngroups = (n + 15) / 16;
    const int nblk = (int)((ngroups + kScanGroupsPerBlock - 1) / kScanGroupsPerBlock);
    uint32_t *block_sums = q.offsets + ngroups;
    uint32_t *block_prefix = block_sums + nblk;
    hipLaunchKernelGGL(queue_scan_local_kernel, dim3(nblk), dim3(kScanBlock), 0, stream,
                       (const uint16_t *)q.mask, ngroups, q.offsets, block_sums);
    hipLaunchKernelGGL(queue_scan_blocks_kernel, dim3(1), dim3(1024), 0, stream,
                       (const uint32_t *)block_sums, nblk, block_prefix, q.count);
    hipLaunchKernelGGL(queue_scatter_kernel, dim3((unsigned)((ngroups + 255) / 256)), dim3(256), 0,
                       stream, (const uint16_t *)q.mask, (const uint32_t *)q.offsets,
                       (const uint32_t *)block_prefix, ngroups, q.idx);
    return hipGetLastError();
}

}  // namespace fab
