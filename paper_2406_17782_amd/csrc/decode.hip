// Neural shading (Sec. 4.2 decoder, Sec. 4.3 rendering) on MFMA.
//
// Each wavefront keeps the whole packed decoder in registers and walks
// 16-pixel tiles of the G-buffer.  Per tile it loads the pixels' SoA fields,
// builds the spatial encoding (8 Fourier frequencies of the pattern-tiled uv,
// one-blob of the footprint size) directly in the MFMA B-operand layout, runs
// the four dense layers as 16x16xK MFMA tiles (M = neurons, N = pixels) with
// the per-fabric first-layer bias c_f (latent folded in) read from LDS, and
// finally decodes and albedo-composes the four components (Eq. (8)).  A
// layer's accumulators feed the next layer's B operand in place (see the slot
// convention in common.hpp), so no data moves between lanes or through LDS
// between layers.
//
// With fallback routing, pixels outside the network's training range are
// shaded in the same call by the analytic footprint filter: the shading
// launch marks them (one bit per pixel), a fixed-order compaction queues
// them in pixel order, and a filter launch shades the queue.
#include "mlp_tile.hpp"
#include "mlp_tile32.hpp"
#include "shade.hpp"

namespace fab {

namespace {

template <int P, bool RAW, bool HYBRID>
__global__ __launch_bounds__(256) void decode_kernel(
    fabric_gbuffer g, const DevFabric *__restrict__ fabrics, int n_fabrics,
    const float *__restrict__ cfold, const typename Mfma<P>::Frag *__restrict__ frags,
    const f32x4 *__restrict__ bias, FallbackQueue q, float *__restrict__ out,
    unsigned long long *err, int n_tiles)
{
    using T = Tile<P>;
    using Frag = typename T::Frag;
    using S = typename T::S;
    using FM = FeatureMath<P>;

    // LDS: C-operand biases of L2..L4 [kBiasFrags][64 lanes], then per fabric
    // c_f [64], then the staged constants [kFabCopies][n_fabrics][kFabConsts].
    extern __shared__ f32x4 smem4[];
    f32x4 *s_bias = smem4;
    float *s_cf = (float *)(smem4 + kBiasFrags * 64);
    float *s_fc = s_cf + n_fabrics * 64;
    for (int k = threadIdx.x; k < kBiasFrags * 64; k += blockDim.x)
        s_bias[k] = bias[k];
    for (int k = threadIdx.x; k < n_fabrics * 64; k += blockDim.x)
        s_cf[k] = cfold[k];
    stage_fabric_consts(fabrics, n_fabrics, s_fc);
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int grp = lane >> 4;
    const int col = lane & 15;

    // The whole decoder stays in registers for the wave's lifetime.
    Frag A[S::NFRAG];
#pragma unroll
    for (int q = 0; q < S::NFRAG; q++)
        A[q] = frags[q * 64 + lane];
    auto getA = [&](int q) { return A[q]; };
    auto getBias = [&](int q) { return s_bias[q * 64 + lane]; };

    const int n = (int)g.n;
    const int waves = gridDim.x * (blockDim.x >> 6);
    const int wave_id = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);

    for (int tile = wave_id; tile < n_tiles; tile += waves) {
        const int p = tile * 16 + col;
        const bool valid = p < n;
        const int pc = valid ? p : n - 1;
        int fid = g.fabric_id[pc];
        const float u = g.u[pc], v = g.v[pc], r = g.radius[pc];
        const float3 wi = make_float3(g.wi_x[pc], g.wi_y[pc], g.wi_z[pc]);
        const float3 wo = make_float3(g.wo_x[pc], g.wo_y[pc], g.wo_z[pc]);
        const bool fault = pixel_fault(fid, n_fabrics, u, v, r, wi, wo);
        // Only the table index needs a safe value: non-finite inputs stay in
        // their own pixel's column of every MFMA tile and are zeroed on output.
        fid = fault ? 0 : fid;
        const float *fc = s_fc + fab_entry(fid, n_fabrics, wi.z) * kFabConsts;

        float s1[T::NS1];
        T::spatial_slots(u, v, r, fc[0], fc[1], fc[2], fc[3], grp, s1);
        f32x4 cf[4];
#pragma unroll
        for (int mb = 0; mb < 4; mb++)
            cf[mb] = *(const f32x4 *)(s_cf + fid * 64 + 16 * mb + 4 * grp);
        float ang0, ang1;
        angular_slots(grp, wi, wo, &ang0, &ang1);
        f32x4 a1[4], a2[4], a3[4], y;
        T::forward(getA, getBias, cf, s1, ang0, ang1, a1, a2, a3, y);

        // Lanes 0..15 hold y[0..3] of pixel tile*16 + lane.
        const bool oor = HYBRID && !fault && out_of_range(r, wo.z);
        if (grp == 0 && valid && !oor) {
            if (RAW) {
#pragma unroll
                for (int c = 0; c < 4; c++)
                    out[c * n + p] = fault ? 0.0f : y[c];
            } else {
                float rgb[3];
                compose_rgb<FM>(y[0], y[1], y[2], y[3], fc, rgb);
#pragma unroll
                for (int c = 0; c < 3; c++)
                    out[c * n + p] = fault ? 0.0f : rgb[c];
            }
        }
        const unsigned long long bad = __ballot(grp == 0 && valid && fault);
        if (lane == 0 && bad)
            atomicAdd(err, (unsigned long long)__popcll(bad));

        // Out-of-range pixels are marked for the footprint filter.
        if (HYBRID)
            queue_mark16((uint32_t)__ballot(grp == 0 && valid && oor), tile, q, lane);
    }
}

// Neural shading on 32x32x16 MFMA tiles (bf16 / fp16): 32 pixels per wave
// iteration, two lane groups per pixel.  Same stages as decode_kernel.
// Each lane group loads only the fields it uses (HalfPix), one tile ahead of
// the one it shades.
template <int P, bool HYBRID>
__global__ __launch_bounds__(256) void decode32_kernel(
    fabric_gbuffer g, const DevFabric *__restrict__ fabrics, int n_fabrics,
    const float *__restrict__ cfold, const typename Mfma<P>::Frag *__restrict__ frags,
    const float *__restrict__ bias2, const f32x4 *__restrict__ bias4,
    const float *__restrict__ cf_scale, FallbackQueue q, float *__restrict__ out,
    unsigned long long *err, int n_tiles)
{
    using T = Tile32<P>;
    using Frag = typename T::Frag;
    using S = typename T::S;
    using FM = FeatureMath<P>;

    // LDS: L2's bias [64], then per fabric c_f [64], then the staged
    // constants [kFabCopies][n_fabrics][kFabConsts].  Both biases are read as
    // the C operands' rows of the lane's group: broadcast reads.
    extern __shared__ f32x4 smem4[];
    float *s_b2 = (float *)smem4;
    float *s_cf = s_b2 + 64;
    float *s_fc = s_cf + n_fabrics * 64;
    for (int k = threadIdx.x; k < 64; k += blockDim.x)
        s_b2[k] = bias2[k];
    for (int k = threadIdx.x; k < n_fabrics * 64; k += blockDim.x)
        s_cf[k] = cfold[k] * cf_scale[k & 63];
    stage_fabric_consts(fabrics, n_fabrics, s_fc);
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int grp = lane >> 5;
    const uint32_t dmask = half_dir_mask(grp);
    const int col = lane & 31;

    Frag A[S::NFRAG];
#pragma unroll
    for (int q = 0; q < S::NFRAG; q++)
        A[q] = frags[q * 64 + lane];
    auto getA = [&](int q) { return A[q]; };
    const f32x4 b4 = bias4[lane];

    const int n = (int)g.n;
    const int waves = gridDim.x * (blockDim.x >> 6);
    const int wave_id = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const HalfPlanes hp = half_planes(g, grp);
    // Pixel of this lane in tile t, clamped for the prefetch past the last
    // tile (t * 32 stays below 2^31: n is at most INT32_MAX / 16 and t less
    // than n_tiles + waves).
    auto tile_px = [&](int t) { return min(t * 32 + col, n - 1); };

    auto shade_tile = [&](const HalfPix &cur, int tile) {
        const int p = tile * 32 + col;
        const bool valid = p < n;
        const unsigned long long fmask = pair_mask(half_fault(cur, n_fabrics, dmask));
        const bool fault = __builtin_amdgcn_inverse_ballot_w64(fmask);
        // Out-of-range rule (r > 1 cell or wo.z < 0.05), decided before the
        // MFMA chain so that no pixel field stays live through it.
        const bool oor = HYBRID && !fault &&
                         pair_any(cur.r > 1.0f || (grp == 1 && cur.xz < 0.05f));
        // Only the table index needs a safe value: non-finite inputs stay in
        // their own pixel's column of every MFMA tile and are zeroed on output.
        const int fid = fault ? 0 : cur.fid;
        // Group 0 holds wi and composes; group 1 only reads the periods.
        const float *fc = s_fc + fab_entry(fid, n_fabrics, grp ? 1.0f : cur.xz) * kFabConsts;

        float s1[kL1Slots32];
        T::spatial_slots(cur.uv, cur.uv, cur.r, fc[0], fc[1], fc[2], fc[3], grp, s1);
        f32x16 cf[2], b2[2];
#pragma unroll
        for (int mb = 0; mb < 2; mb++)
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int row = 32 * mb + 8 * q + 4 * grp;
                const f32x4 c4 = *(const f32x4 *)(s_cf + fid * 64 + row);
                const f32x4 bq = *(const f32x4 *)(s_b2 + row);
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    cf[mb][4 * q + i] = c4[i];
                    b2[mb][4 * q + i] = bq[i];
                }
            }
        // L3 extra inputs: group 0 wi, group 1 (wo.x, wo.y, 1 for the bias).
        const float x2 = grp ? 1.0f : cur.xz;
        const f32x4 y = T::forward(getA, cf, b2, b4, s1, cur.x0, cur.x1, x2);

        // Lanes 0..31 hold y[0..3] of pixel tile*32 + lane.
        if (grp == 0 && valid && !oor) {
            float rgb[3];
            compose_rgb<FM>(y[0], y[1], y[2], y[3], fc, rgb);
#pragma unroll
            for (int c = 0; c < 3; c++)
                plane_store(out, c * n + p, fault ? 0.0f : rgb[c]);
        }
        // Faulted pixels of the tile, counted once (lane group 0's bits).
        const unsigned long long bad = fmask & __ballot(valid) & 0xffffffffull;
        if (lane == 0 && bad)
            atomicAdd(err, (unsigned long long)__popcll(bad));
        if (HYBRID)
            queue_mark32((uint32_t)__ballot(grp == 0 && valid && oor), tile, q, lane);
    };

    // The next tile's fields are loaded while this one is shaded (loading
    // two tiles ahead measured no faster).
    HalfPix nxt = load_half(g, hp, tile_px(wave_id));
    for (int tile = wave_id; tile < n_tiles; tile += waves) {
        const HalfPix cur = nxt;
        nxt = load_half(g, hp, tile_px(tile + waves));
        shade_tile(cur, tile);
    }
}

// Scale exponents of the 32-pixel layout's hidden neurons (BF16; zero for
// FP16): e such that 2^e exceeds an upper bound U of the neuron's
// pre-activation over every input, U from the weights as the image uses
// them and the encoded fabrics' first-layer biases:
//   U1_i = max_f c_f,i + sum_j |W1s_ij|          (spatial features in [-1, 1])
//   U2_i = b2_i + sum_j max(W2_ij, 0) max(U1_j, 0)            (h1 >= 0)
//   U3_i = b3_i + sum_j max(W3_ij, 0) max(U2_j, 0) + sum_a |W3a_ia|
// (the angular inputs are unit-vector components), with a margin of 1 %
// for the rounding of weights and sums.  A neuron whose bound is not
// positive is never active (e = 0).  One block of 64 threads.
template <int P>
__global__ __launch_bounds__(64) void scale32_kernel(const float *__restrict__ params,
                                                     const float *__restrict__ cfold, int n_fabrics,
                                                     int *__restrict__ exps, float *__restrict__ cf_scale)
{
    __shared__ float U[64];
    const int i = threadIdx.x;
    auto expo = [](float u) {
        if (!(u > 0.0f) || P != FABRIC_BF16)
            return 0;
        int e = (int)floorf(log2f(1.01f * u)) + 1;
        return min(max(e, -60), 60);
    };
    float c = -INFINITY;
    for (int f = 0; f < n_fabrics; f++)
        c = fmaxf(c, cfold[f * 64 + i]);
    float u = c;
    for (int j = 0; j < kFeat; j++)
        u += fabsf(params[kOffW1 + i * 72 + kLatent + j]);
    int e = expo(u);
    exps[i] = e;
    cf_scale[i] = ldexpf(1.0f, -e);
    U[i] = fmaxf(u, 0.0f);
    __syncthreads();
    u = params[kOffB2 + i];
    for (int j = 0; j < 64; j++)
        u += fmaxf(params[kOffW2 + i * 64 + j], 0.0f) * U[j];
    __syncthreads();
    U[i] = fmaxf(u, 0.0f);
    exps[64 + i] = expo(u);
    __syncthreads();
    u = params[kOffB3 + i];
    for (int j = 0; j < 64; j++)
        u += fmaxf(params[kOffW3 + i * 69 + j], 0.0f) * U[j];
    for (int a = 0; a < 5; a++)
        u += fabsf(params[kOffW3 + i * 69 + 64 + a]);
    exps[128 + i] = expo(u);
}

// Image of the 32-pixel layout from FP32 decoder parameters and the scale
// exponents of scale32_kernel: hidden neuron i of layer l is scaled by
// 2^-e_l,i (its weights, bias and, for L1, c_f) and the next layer's
// weights of that input by 2^e_l,i.
template <int P>
__global__ void pack_decoder32_kernel(const float *__restrict__ params, const int *__restrict__ exps,
                                      typename Mfma<P>::Frag *__restrict__ frags,
                                      float *__restrict__ bias2, f32x4 *__restrict__ bias4)
{
    using M = Mfma<P>;
    using S = DecShape32<8>;
    const int *e1 = exps, *e2 = exps + 64, *e3 = exps + 128;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < S::NFRAG * 64) {
        const int fr = idx / 64, lane = idx % 64, row = lane & 31, grp = lane >> 5;
        int layer, mb, ks;
        if (fr < S::FRAG_L2) { layer = 1; mb = fr / S::KS1; ks = fr % S::KS1; }
        else if (fr < S::FRAG_L3) { layer = 2; mb = (fr - S::FRAG_L2) / S::KS2; ks = (fr - S::FRAG_L2) % S::KS2; }
        else if (fr < S::FRAG_L4) { layer = 3; mb = (fr - S::FRAG_L3) / S::KS3; ks = (fr - S::FRAG_L3) % S::KS3; }
        else { layer = 4; mb = 0; ks = fr - S::FRAG_L4; }
        const int m = 32 * mb + row;
        typename M::Frag f = M::zero();
        for (int j = 0; j < 8; j++) {
            const int c = ks * 8 + j;
            float w = 0.0f;
            if (layer == 1) {
                const int feat = l1_feature32(grp, c);
                if (feat >= 0) w = ldexpf(params[kOffW1 + m * 72 + kLatent + feat], -e1[m]);
            } else if (layer == 2) {
                if (c < kChain32) {
                    const int nj = chain32_neuron(grp, c);
                    w = ldexpf(params[kOffW2 + m * 64 + nj], e1[nj] - e2[m]);
                }
            } else if (layer == 3) {
                if (c < kChain32) {
                    const int nj = chain32_neuron(grp, c);
                    w = ldexpf(params[kOffW3 + m * 69 + nj], e2[nj] - e3[m]);
                } else if (c < kL3Slots32) {
                    const int a = l3_extra32(grp, c - kChain32);
                    if (a == 5) w = ldexpf(params[kOffB3 + m], -e3[m]);
                    else if (a >= 0) w = ldexpf(params[kOffW3 + m * 69 + 64 + a], -e3[m]);
                }
            } else {
                // 16x16x32 operand: lane l holds A[row l%16][K block l/16];
                // rows 0..3 read K blocks 0 and 2 (pixels 0..15), rows 4..7
                // K blocks 1 and 3 (pixels 16..31), of lane group kb/2.
                const int r16 = lane & 15, kb = lane >> 4;
                const int out = r16 < 4 && (kb & 1) == 0 ? r16
                              : (r16 >= 4 && r16 < 8 && (kb & 1) == 1 ? r16 - 4 : -1);
                if (out >= 0) {
                    const int nj = chain32_neuron(kb >> 1, c);
                    w = ldexpf(params[kOffW4 + out * 64 + nj], e3[nj]);
                }
            }
            M::set(f, j, w);
        }
        frags[idx] = f;
    }
    if (idx < 64)
        bias2[idx] = ldexpf(params[kOffB2 + idx], -e2[idx]);
    if (idx < 64) {
        // 16x16 C operand: lanes 0..31 hold rows 0..3 / 4..7, the four outputs
        // of their own pixel.
        f32x4 b;
        for (int i = 0; i < 4; i++)
            b[i] = idx < 32 ? params[kOffB4 + i] : 0.0f;
        bias4[idx] = b;
    }
}

// Fill the fragment image of precision P from FP32 decoder parameters.
template <int P>
__global__ void pack_decoder_kernel(const float *__restrict__ params,
                                    typename Mfma<P>::Frag *__restrict__ frags,
                                    f32x4 *__restrict__ bias)
{
    using M = Mfma<P>;
    using S = DecShape<M::KPL>;
    constexpr int KPL = M::KPL;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < S::NFRAG * 64) {
        const int fr = idx / 64, lane = idx % 64;
        const int row = lane & 15, grp = lane >> 4;
        int layer, mb, ks;
        if (fr < S::FRAG_L2) { layer = 1; mb = (fr - S::FRAG_L1) / S::KS1; ks = (fr - S::FRAG_L1) % S::KS1; }
        else if (fr < S::FRAG_L3) { layer = 2; mb = (fr - S::FRAG_L2) / S::KS2; ks = (fr - S::FRAG_L2) % S::KS2; }
        else if (fr < S::FRAG_L4) { layer = 3; mb = (fr - S::FRAG_L3) / S::KS3; ks = (fr - S::FRAG_L3) % S::KS3; }
        else { layer = 4; mb = 0; ks = fr - S::FRAG_L4; }
        const int m = 16 * mb + row;
        typename M::Frag f = M::zero();
        for (int j = 0; j < KPL; j++) {
            const int c = ks * KPL + j;
            float w = 0.0f;
            if (layer == 1) {
                int feat = l1_feature(grp, c);
                if (feat >= 0) w = params[kOffW1 + m * 72 + kLatent + feat];
            } else if (layer == 2) {
                if (c < kChainSlots) w = params[kOffW2 + m * 64 + chain_neuron(grp, c)];
            } else if (layer == 3) {
                if (c < kChainSlots) {
                    w = params[kOffW3 + m * 69 + chain_neuron(grp, c)];
                } else if (c < kL3Slots) {
                    int a = l3_angular(grp, c - kChainSlots);
                    if (a >= 0) w = params[kOffW3 + m * 69 + 64 + a];
                }
            } else {
                if (m < 4 && c < kChainSlots) w = params[kOffW4 + m * 64 + chain_neuron(grp, c)];
            }
            M::set(f, j, w);
        }
        frags[idx] = f;
    }
    if (idx < kBiasFrags * 64) {
        const int bf = idx / 64, lane = idx % 64, grp = lane >> 4;
        f32x4 b;
        for (int i = 0; i < 4; i++) {
            float val;
            if (bf < 4) val = params[kOffB2 + 16 * bf + 4 * grp + i];
            else if (bf < 8) val = params[kOffB3 + 16 * (bf - 4) + 4 * grp + i];
            else val = (4 * grp + i) < 4 ? params[kOffB4 + 4 * grp + i] : 0.0f;
            b[i] = val;
        }
        bias[idx] = b;
    }
}

__global__ void fold_latents_kernel(const float *__restrict__ params,
                                    const float *__restrict__ latents, int n_fabrics,
                                    float *__restrict__ cfold)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_fabrics * 64)
        return;
    const int f = idx / 64, o = idx % 64;
    float acc = params[kOffB1 + o];
    for (int k = 0; k < kLatent; k++)
        acc = fmaf(params[kOffW1 + o * 72 + k], latents[f * kLatent + k], acc);
    cfold[idx] = acc;
}

// Parts of the 32-pixel layout's image (see Tile32).
struct Image32 {
    void *frags;
    float *b2;
    f32x4 *b4;
    int *exps;
    float *cf_scale;
};
inline Image32 image32_parts(const void *image)
{
    Image32 im;
    char *base = (char *)image;
    im.frags = base;
    im.b2 = (float *)(base + (size_t)DecShape32<8>::NFRAG * 64 * 16);
    im.b4 = (f32x4 *)(im.b2 + 64);
    im.exps = (int *)(im.b4 + 64);
    im.cf_scale = (float *)(im.exps + 3 * 64);
    return im;
}

size_t image32_bytes()
{
    return (size_t)DecShape32<8>::NFRAG * 64 * 16 + (size_t)64 * sizeof(float) +
           (size_t)64 * sizeof(f32x4) + (size_t)3 * 64 * sizeof(int) + (size_t)64 * sizeof(float);
}

template <int P>
hipError_t pack32(const float *params, const float *cfold, int n_fabrics, void *image,
                  hipStream_t stream)
{
    using M = Mfma<P>;
    const Image32 im = image32_parts(image);
    hipLaunchKernelGGL(scale32_kernel<P>, dim3(1), dim3(64), 0, stream, params, cfold, n_fabrics,
                       im.exps, im.cf_scale);
    const int total = DecShape32<8>::NFRAG * 64;
    hipLaunchKernelGGL(pack_decoder32_kernel<P>, dim3((total + 255) / 256), dim3(256), 0, stream,
                       params, (const int *)im.exps, (typename M::Frag *)im.frags, im.b2, im.b4);
    return hipGetLastError();
}

template <int P, bool HYBRID>
hipError_t decode32(const fabric_gbuffer &g, const DevFabric *fabrics, int n_fabrics,
                    const float *cfold, const void *image, FallbackQueue q, float *out,
                    unsigned long long *err, hipStream_t stream)
{
    using M = Mfma<P>;
    const Image32 im = image32_parts(image);
    const int n_tiles = (int)((g.n + 31) / 32);
    int blocks = (n_tiles + 3) / 4;
    const int cap = device_cus() * 2;
    if (blocks > cap)
        blocks = cap;
    const size_t lds = (size_t)64 * sizeof(float) +
                       (size_t)n_fabrics * (64 + kFabCopies * kFabConsts) * sizeof(float);
    hipLaunchKernelGGL((decode32_kernel<P, HYBRID>), dim3(blocks), dim3(256), lds, stream, g,
                       fabrics, n_fabrics, cfold, (const typename M::Frag *)im.frags, im.b2,
                       im.b4, im.cf_scale, q, out, err, n_tiles);
    return hipGetLastError();
}

template <int P> size_t image_bytes()
{
    using M = Mfma<P>;
    using S = DecShape<M::KPL>;
    return (size_t)S::NFRAG * 64 * sizeof(typename M::Frag) + (size_t)kBiasFrags * 64 * sizeof(f32x4);
}

template <int P> hipError_t pack(const float *params, void *image, hipStream_t stream)
{
    using M = Mfma<P>;
    using S = DecShape<M::KPL>;
    auto *frags = (typename M::Frag *)image;
    auto *bias = (f32x4 *)((char *)image + (size_t)S::NFRAG * 64 * sizeof(typename M::Frag));
    const int total = S::NFRAG * 64 > kBiasFrags * 64 ? S::NFRAG * 64 : kBiasFrags * 64;
    hipLaunchKernelGGL(pack_decoder_kernel<P>, dim3((total + 255) / 256), dim3(256), 0, stream,
                       params, frags, bias);
    return hipGetLastError();
}


template <int P, bool RAW, bool HYBRID>
hipError_t decode(const fabric_gbuffer &g, const DevFabric *fabrics, int n_fabrics,
                  const float *cfold, const void *image, FallbackQueue q, float *out,
                  unsigned long long *err, hipStream_t stream)
{
    using M = Mfma<P>;
    using S = DecShape<M::KPL>;
    const auto *frags = (const typename M::Frag *)image;
    const auto *bias =
        (const f32x4 *)((const char *)image + (size_t)S::NFRAG * 64 * sizeof(typename M::Frag));
    const int n_tiles = (int)((g.n + 15) / 16);
    int blocks = (n_tiles + 3) / 4;
    const int cap = device_cus() * 2;
    if (blocks > cap)
        blocks = cap;
    const size_t lds = (size_t)kBiasFrags * 64 * sizeof(f32x4) +
                       (size_t)n_fabrics * (64 + kFabCopies * kFabConsts) * sizeof(float);
    hipLaunchKernelGGL((decode_kernel<P, RAW, HYBRID>), dim3(blocks), dim3(256), lds,
                       stream, g, fabrics, n_fabrics, cfold, frags, bias, q, out, err, n_tiles);
    return hipGetLastError();
}

}  // namespace

int device_cus()
{
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
    }
    return cus;
}

size_t decoder_image_bytes(int prec)
{
    switch (prec) {
    case FABRIC_FP32: return image_bytes<FABRIC_FP32>();
    case FABRIC_BF16: return image_bytes<FABRIC_BF16>();
    case FABRIC_FP16: return image_bytes<FABRIC_FP16>();
    default: return 0;
    }
}

hipError_t launch_pack_decoder(int prec, const float *dec_params, void *image, hipStream_t stream)
{
    switch (prec) {
    case FABRIC_FP32: return pack<FABRIC_FP32>(dec_params, image, stream);
    case FABRIC_BF16: return pack<FABRIC_BF16>(dec_params, image, stream);
    case FABRIC_FP16: return pack<FABRIC_FP16>(dec_params, image, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fold_latents(const float *dec_params, const float *latents, int n_fabrics,
                               float *cfold, hipStream_t stream)
{
    const int total = n_fabrics * 64;
    hipLaunchKernelGGL(fold_latents_kernel, dim3((total + 255) / 256), dim3(256), 0, stream,
                       dec_params, latents, n_fabrics, cfold);
    return hipGetLastError();
}

size_t shade_image_bytes(int prec)
{
    if (prec == FABRIC_FP8_E4M3)
        return f8_image_bytes();
    return (prec == FABRIC_BF16 || prec == FABRIC_FP16) ? image32_bytes() : decoder_image_bytes(prec);
}

hipError_t launch_pack_shade(int prec, const float *dec_params, const float *cfold, int n_fabrics,
                             void *image, hipStream_t stream)
{
    switch (prec) {
    case FABRIC_BF16: return pack32<FABRIC_BF16>(dec_params, cfold, n_fabrics, image, stream);
    case FABRIC_FP16: return pack32<FABRIC_FP16>(dec_params, cfold, n_fabrics, image, stream);
    default: return launch_pack_decoder(prec, dec_params, image, stream);
    }
}

hipError_t launch_decode(int prec, bool raw, const fabric_gbuffer &g, const DevFabric *fabrics,
                         int n_fabrics, const float *cfold, const void *image,
                         int fallback_samples, uint64_t seed, VisArgs vis, FallbackQueue q,
                         float *out, unsigned long long *err, hipStream_t stream)
{
    if (g.n == 0)
        return hipSuccess;
    const bool hybrid = !raw && fallback_samples > 0;
    hipError_t e = hipSuccess;
    if (prec == FABRIC_FP8_E4M3)
        e = raw ? hipErrorInvalidValue
                : launch_decode_f8(g, fabrics, n_fabrics, cfold, image, hybrid, q, out, err, stream);
    else if (!raw && prec == FABRIC_BF16)
        // Shading in bf16 / fp16 runs on 32-pixel tiles (image from
        // launch_pack_shade); the raw forward and fp32 on 16-pixel tiles.
        e = hybrid ? decode32<FABRIC_BF16, true>(g, fabrics, n_fabrics, cfold, image, q, out, err, stream)
                   : decode32<FABRIC_BF16, false>(g, fabrics, n_fabrics, cfold, image, q, out, err, stream);
    else if (!raw && prec == FABRIC_FP16)
        e = hybrid ? decode32<FABRIC_FP16, true>(g, fabrics, n_fabrics, cfold, image, q, out, err, stream)
                   : decode32<FABRIC_FP16, false>(g, fabrics, n_fabrics, cfold, image, q, out, err, stream);
    else if (prec == FABRIC_FP32)
        e = raw ? decode<FABRIC_FP32, true, false>(g, fabrics, n_fabrics, cfold, image, q, out, err, stream)
                : hybrid ? decode<FABRIC_FP32, false, true>(g, fabrics, n_fabrics, cfold, image, q, out, err, stream)
                         : decode<FABRIC_FP32, false, false>(g, fabrics, n_fabrics, cfold, image, q, out, err, stream);
    else if (raw && prec == FABRIC_BF16)
        e = decode<FABRIC_BF16, true, false>(g, fabrics, n_fabrics, cfold, image, q, out, err, stream);
    else
        e = hipErrorInvalidValue;
    if (e != hipSuccess || !hybrid)
        return e;
    if ((e = launch_queue_build(q, g.n, stream)) != hipSuccess)
        return e;
    return launch_gt_filter_queue(g, fabrics, fallback_samples, seed, vis, q, out, stream);
}

}  // namespace fab
