// The decoder at the paper's own form (Sec. 4.2 "Decoder"): latent 64; the
// footprint's position and size one-blob encoded to 24 channels; spatial
// fusion by two FC layers; an angular decoder of five FC layers over
// [spatial feature, wi.xyz, wo.xy] whose second and third layers form a
// residual block (the block's input added before its last activation);
// leaky ReLU (slope 0.01) after every layer but the output.  Width 64.
//
// BF16 operands on 32x32x16 MFMA with FP32 accumulation, 32-pixel tiles in
// the layout of the config decoder's shading kernel (lane group g = l/32
// owns chained neurons 32 mb + 8 (r/4) + 4 g + r%4; one layer's output is
// the next layer's B operand without data movement).  The 58 weight
// fragments (58 KB) stay in LDS and are read before each MFMA, which leaves
// the registers to four waves per SIMD; each layer's bias rides in a K slot
// that holds 1 (the first extra slot of lane group 0): layer F1's bias is
// folded with the latent into the per-fabric C operand c_f, A1's extra slots
// carry wi.xyz / wo.xy / 1 as in the config decoder, A3's C operand is the
// residual x, A5's bias is added after the MFMA.
#include "kernels.hpp"
#include "mlp_tile32.hpp"
#include "model.hpp"
#include "paper_net.hpp"
#include "paper_tile.hpp"
#include "shade.hpp"

namespace fab {

namespace {


template <int P>
__global__ void pack_paper_kernel(const float *__restrict__ params,
                                  typename Mfma<P>::Frag *__restrict__ frags,
                                  f32x4 *__restrict__ b5, int fused)
{
    using M = Mfma<P>;
    using Frag = typename M::Frag;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < kPFrags * 64) {
        const int fr = idx / 64, lane = idx % 64, row = lane & 31, grp = lane >> 5;
        int layer = 0;
        while (layer + 1 < kPLayers && fr >= p_first(layer + 1))
            layer++;
        const int local = fr - p_first(layer);
        const int mb = local / p_ks(layer), ks = local % p_ks(layer);
        const int m = 32 * mb + row;
        Frag f = M::zero();
        for (int j = 0; j < 8; j++) {
            const int c = ks * 8 + j;
            float w = 0.0f;
            if (layer == kF1) {
                const int ch = p_blob_channel(grp, c);
                const int a = fused ? -1 : p_f1_angular(grp, c);
                if (ch >= 0) w = params[kPOffWF1 + m * kPX1 + kPLat + ch];
                else if (a >= 0) w = params[kPOffWA1 + m * kPXA1 + 64 + a];
            } else if (layer == kA1) {
                if (c < kChain32) {
                    w = params[kPOffWA1 + m * kPXA1 + chain32_neuron(grp, c)] *
                        paper_weight_scale(P, kA1);
                } else if (c < kL3Slots32) {
                    const int a = l3_extra32(grp, c - kChain32);
                    if (a == 5) w = params[kPOffBA1 + m];
                    else if (a >= 0 && fused) w = params[kPOffWA1 + m * kPXA1 + 64 + a];
                }
            } else if (layer == kA5) {
                if (m < 4 && c < kChain32)
                    w = params[kPOffWA5 + m * 64 + chain32_neuron(grp, c)] * paper_weight_scale(P, kA5);
            } else {
                const int offw = layer == kF2 ? kPOffWF2 : layer == kA2 ? kPOffWA2
                                 : layer == kA3 ? kPOffWA3 : kPOffWA4;
                const int offb = layer == kF2 ? kPOffBF2 : layer == kA2 ? kPOffBA2
                                 : layer == kA3 ? kPOffBA3 : kPOffBA4;
                if (c < kChain32)
                    w = params[offw + m * 64 + chain32_neuron(grp, c)] * paper_weight_scale(P, layer);
                else if (c == kChain32 && grp == 0)
                    w = params[offb + m] * paper_bias_scale(P, layer);
            }
            M::set(f, j, w);
        }
        frags[idx] = f;
    }
    if (idx < 64) {
        f32x4 b;
        for (int i = 0; i < 4; i++)
            b[i] = (idx >> 5) == 0 ? params[kPOffBA5 + i] : 0.0f;
        b5[idx] = b;
    }
}

// c_f = WF1[:, 0:64] z_f + bF1 for every fabric: cfold[n_fabrics][64].
__global__ void fold_paper_kernel(const float *__restrict__ params,
                                  const float *__restrict__ latents, int n_fabrics,
                                  float *__restrict__ cfold)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_fabrics * 64)
        return;
    const int f = idx / 64, o = idx % 64;
    float acc = params[kPOffBF1 + o];
    for (int k = 0; k < kPLat; k++)
        acc = fmaf(params[kPOffWF1 + o * kPX1 + k], latents[f * kPLat + k], acc);
    cfold[idx] = acc;
}

// Shading of T tiles per wave iteration (T x 32 pixels).
template <int P, int WAVES, int T, bool RAW, bool FUSED>
__global__ __launch_bounds__(64 * WAVES) void decode_paper_kernel(
    fabric_gbuffer g, const DevFabric *__restrict__ fabrics, int n_fabrics,
    const float *__restrict__ cfold, const typename Mfma<P>::Frag *__restrict__ frags,
    const f32x4 *__restrict__ bias5, float *__restrict__ out, unsigned long long *err, int n_tiles)
{
    using PT = PaperTile<P>;
    using M = typename PT::M;
    using Frag = typename PT::Frag;
    using FM = FeatureMath<P>;
    // LDS: the 58 weight fragments, then per fabric c_f [64], then the staged
    // constants [kFabCopies][n_fabrics][kFabConsts].
    extern __shared__ f32x4 smem4[];
    Frag *s_w = (Frag *)smem4;
    float *s_cf = (float *)(smem4 + kPFrags * 64);
    float *s_fc = s_cf + n_fabrics * 64;
    for (int k = threadIdx.x; k < kPFrags * 64; k += blockDim.x)
        s_w[k] = frags[k];
    for (int k = threadIdx.x; k < n_fabrics * 64; k += blockDim.x)
        s_cf[k] = cfold[k];
    stage_fabric_consts(fabrics, n_fabrics, s_fc);
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int grp = lane >> 5;
    const uint32_t dmask = half_dir_mask(grp);
    const int col = lane & 31;
    const f32x4 b5 = bias5[lane];
    // The bias K step of the chain layers: 1 in slot 32 of lane group 0.
    f32x8 one8 = {grp == 0 ? 1.0f : 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    const Frag bias_b = M::from8(one8);

    const int n = (int)g.n;
    const int waves = gridDim.x * WAVES;
    const int wave_id = blockIdx.x * WAVES + (threadIdx.x >> 6);
    const HalfPlanes hp = half_planes(g, grp);
    // Wave w takes tiles T w + t, T w + t + T waves, ...; indices past the
    // end load a clamped pixel and store nothing.
    auto tile_px = [&](int t) { return min(t * 32 + col, n - 1); };

    auto shade = [&](const HalfPix (&cur)[T], int tile0) {
        // An offset the compiler cannot see through, so that the weight
        // reads stay inside the loop instead of being hoisted into
        // registers for all tiles (58 fragments would not fit).
        int wofs = 0;
        asm volatile("" : "+s"(wofs));
        const Frag *s_wt = s_w + wofs;

        int p[T], fid[T], entry[T];
        bool valid[T], fault[T];
        f32x16 a[T][2];
        {
            Frag B1[T][2];
#pragma unroll
            for (int t = 0; t < T; t++) {
                p[t] = (tile0 + t) * 32 + col;
                valid[t] = tile0 + t < n_tiles && p[t] < n;
                fault[t] = pair_any(half_fault(cur[t], n_fabrics, dmask));
                fid[t] = fault[t] ? 0 : cur[t].fid;
                entry[t] = fab_entry(fid[t], n_fabrics, grp ? 1.0f : cur[t].xz);
                const float *fc = s_fc + entry[t] * kFabConsts;
                // F1: one-blob slots; C operand c_f.
                // Without fusion, four more slots carry the angular inputs.
                float s1[FUSED ? kPSlots1 : kPSlots1 + 4];
                const float per = grp ? fc[1] : fc[0], iper = grp ? fc[3] : fc[2];
                paper_slots<P, RAW>(wrap_period(cur[t].uv, per, iper), iper, cur[t].r, grp, s1);
                if (!FUSED) {
                    s1[kPSlots1] = cur[t].x0;
                    s1[kPSlots1 + 1] = cur[t].x1;
                    s1[kPSlots1 + 2] = grp ? 0.0f : cur[t].xz;
                }
                B1[t][0] = PT::frag_of(s1, 0, false);
                B1[t][1] = PT::frag_of(s1, 1, false);
#pragma unroll
                for (int mb = 0; mb < 2; mb++)
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        const f32x4 c4 =
                            *(const f32x4 *)(s_cf + fid[t] * 64 + 32 * mb + 8 * q + 4 * grp);
#pragma unroll
                        for (int i = 0; i < 4; i++)
                            a[t][mb][4 * q + i] = c4[i];
                    }
            }
            PT::template dense_lds<T, 2, 2>(s_wt, p_first(kF1), B1, a, lane);
        }
        // The chained B operand (with the previous layer's activation fused
        // into the packing when `act`) and its bias step.
        auto chain_in = [&](Frag (&B)[T][5], bool act) {
#pragma unroll
            for (int t = 0; t < T; t++) {
                Frag B4[4];
                PT::chain_b(a[t], B4, act);
#pragma unroll
                for (int ks = 0; ks < 4; ks++)
                    B[t][ks] = B4[ks];
                B[t][4] = bias_b;
            }
        };
        auto chain_layer = [&](int layer, bool act) {
            Frag B[T][5];
            chain_in(B, act);
#pragma unroll
            for (int t = 0; t < T; t++)
                a[t][0] = a[t][1] = f32x16{};
            PT::template dense_lds<T, 2, 5>(s_wt, p_first(layer), B, a, lane);
        };
        chain_layer(kF2, true);                   // spatial feature
        // A1: [spatial feature, wi.xyz | wo.xy, 1].
        {
            Frag B[T][5];
#pragma unroll
            for (int t = 0; t < T; t++) {
                float v[kL3Slots32];
#pragma unroll
                for (int c = 0; c < kChain32; c++)
                    v[c] = a[t][c >> 4][c & 15];
                v[32] = cur[t].x0;
                v[33] = cur[t].x1;
                v[34] = grp ? 1.0f : cur[t].xz;
#pragma unroll
                for (int ks = 0; ks < 5; ks++)
                    B[t][ks] = PT::frag_of(v, ks, ks < 4);
                a[t][0] = a[t][1] = f32x16{};
            }
            PT::template dense_lds<T, 2, 5>(s_wt, p_first(kA1), B, a, lane);
        }
        // The residual block's input, activated in FP32 (it is also A3's C
        // operand); A2 then packs it without a further activation.
        f32x16 x[T][2];
#pragma unroll
        for (int t = 0; t < T; t++) {
            PT::act_acc(a[t]);
            x[t][0] = a[t][0];
            x[t][1] = a[t][1];
        }
        chain_layer(kA2, false);
        // A3 from C operand x: the skip enters before the activation.
        {
            Frag B[T][5];
            chain_in(B, true);
            PT::template dense_lds<T, 2, 5>(s_wt, p_first(kA3), B, x, lane);
#pragma unroll
            for (int t = 0; t < T; t++) {
                a[t][0] = x[t][0];
                a[t][1] = x[t][1];
            }
        }
        chain_layer(kA4, true);
        // A5: four outputs in rows 0..3 (lane group 0), bias added after.
        {
            Frag B[T][4];
#pragma unroll
            for (int t = 0; t < T; t++) {
                PT::chain_b(a[t], B[t], true);
                a[t][0] = f32x16{};
            }
            PT::template dense_lds<T, 1, 4>(s_wt, p_first(kA5), B, a, lane);
        }
#pragma unroll
        for (int t = 0; t < T; t++) {
            if (grp == 0 && valid[t]) {
                float rgb[3];
                compose_rgb<FM>(a[t][0][0] + b5[0], a[t][0][1] + b5[1], a[t][0][2] + b5[2],
                                a[t][0][3] + b5[3], s_fc + entry[t] * kFabConsts, rgb);
#pragma unroll
                for (int c = 0; c < 3; c++)
                    plane_store(out, c * n + p[t], fault[t] ? 0.0f : rgb[c]);
            }
            const unsigned long long bad = __ballot(grp == 0 && valid[t] && fault[t]);
            if (lane == 0 && bad)
                atomicAdd(err, (unsigned long long)__popcll(bad));
        }
    };

    // Loop over this wave's groups of T tiles, loading the next group's
    // fields while the current one is shaded.
    HalfPix nxt[T];
#pragma unroll
    for (int t = 0; t < T; t++)
        nxt[t] = load_half(g, hp, tile_px(T * wave_id + t));
    for (int tile0 = T * wave_id; tile0 < n_tiles; tile0 += T * waves) {
        HalfPix cur[T];
#pragma unroll
        for (int t = 0; t < T; t++) {
            cur[t] = nxt[t];
            nxt[t] = load_half(g, hp, tile_px(tile0 + T * waves + t));
        }
        shade(cur, tile0);
    }
}

// Two tiles per wave iteration share every weight read; 512-thread blocks,
// one per CU, two waves per SIMD.
constexpr int kPaperWaves = 8;
constexpr int kPaperTiles = 2;

}  // namespace

// One image per operand precision: BF16 first, then FP16.
size_t paper_image_bytes()
{
    return 2 * ((size_t)kPFrags * 64 * 16 + (size_t)64 * sizeof(f32x4));
}

template <int P> static void *paper_image_of(void *image)
{
    return (char *)image + (P == FABRIC_FP16 ? paper_image_bytes() / 2 : 0);
}

hipError_t launch_paper_prepare(const float *params, const float *latents, int n_fabrics,
                                bool fused, void *image, float *cfold, hipStream_t stream)
{
    const int blocks = (kPFrags * 64 + 255) / 256;
    {
        using Frag = Mfma<FABRIC_BF16>::Frag;
        auto *frags = (Frag *)paper_image_of<FABRIC_BF16>(image);
        auto *b5 = (f32x4 *)(frags + kPFrags * 64);
        hipLaunchKernelGGL(pack_paper_kernel<FABRIC_BF16>, dim3(blocks), dim3(256), 0, stream,
                           params, frags, b5, fused ? 1 : 0);
    }
    {
        using Frag = Mfma<FABRIC_FP16>::Frag;
        auto *frags = (Frag *)paper_image_of<FABRIC_FP16>(image);
        auto *b5 = (f32x4 *)(frags + kPFrags * 64);
        hipLaunchKernelGGL(pack_paper_kernel<FABRIC_FP16>, dim3(blocks), dim3(256), 0, stream,
                           params, frags, b5, fused ? 1 : 0);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const int total = n_fabrics * 64;
    hipLaunchKernelGGL(fold_paper_kernel, dim3((total + 255) / 256), dim3(256), 0, stream, params,
                       latents, n_fabrics, cfold);
    return hipGetLastError();
}

// FP32 reference shading of the paper-size decoder: one lane per pixel,
// every layer in FP32 from the FP32 masters (latent product included, no
// folding), activation rows in LDS (the weights are the same for every lane:
// scalar loads).  Writes the composed rgb [3][n] and/or the raw outputs
// [4][n]; faulted pixels give zeros and are counted.
constexpr int kRefThreads = 64;
constexpr int kRefStrideA = kPX1 + 1;      // odd strides: one bank per lane
constexpr int kRefStrideB = 64 + 1;

__global__ __launch_bounds__(kRefThreads) void decode_paper_f32_kernel(
    fabric_gbuffer g, const DevFabric *__restrict__ fabrics, int n_fabrics,
    const float *__restrict__ P, const float *__restrict__ lat, int raw, int fused,
    float *__restrict__ out_rgb, float *__restrict__ out_y4, unsigned long long *err)
{
    __shared__ float bufA[kRefThreads * kRefStrideA];
    __shared__ float bufB[kRefThreads * kRefStrideB];
    const int64_t n = g.n;
    const int64_t p = (int64_t)blockIdx.x * kRefThreads + threadIdx.x;
    if (p >= n)
        return;
    const int fid = g.fabric_id[p];
    const float u = g.u[p], v = g.v[p], r = g.radius[p];
    const float3 wi = make_float3(g.wi_x[p], g.wi_y[p], g.wi_z[p]);
    const float3 wo = make_float3(g.wo_x[p], g.wo_y[p], g.wo_z[p]);
    if (pixel_fault(fid, n_fabrics, u, v, r, wi, wo)) {
        for (int c = 0; c < 3 && out_rgb; c++)
            out_rgb[c * n + p] = 0.0f;
        for (int c = 0; c < 4 && out_y4; c++)
            out_y4[c * n + p] = 0.0f;
        atomicAdd(err, 1ull);
        return;
    }
    float *a = bufA + threadIdx.x * kRefStrideA, *b = bufB + threadIdx.x * kRefStrideB;
    const float ang[5] = {wi.x, wi.y, wi.z, wo.x, wo.y};
    // One layer: out[o] = act(W in + bias)[o], act the leaky ReLU (of the
    // sum with the residual `res`, when given) or none (the output layer).
    auto layer = [&](int w_off, int b_off, const float *in, int nin, float *out, int nout,
                     bool act, const float *res) {
        for (int o = 0; o < nout; o++) {
            float acc = P[b_off + o];
            const float *W = P + w_off + o * nin;
#pragma unroll 8
            for (int i = 0; i < nin; i++)
                acc = fmaf(W[i], in[i], acc);
            if (res)
                acc += res[o];
            out[o] = act ? lrelu(acc) : acc;
        }
    };
    for (int k = 0; k < kPLat; k++)
        a[k] = lat[fid * kPLat + k];
    float f[kPBlob];
    blob24(fabrics[fid], u, v, r, raw != 0, f);
    for (int k = 0; k < kPBlob; k++)
        a[kPLat + k] = f[k];
    // F1 (without the fusion stage, A1's angular columns act here instead).
    for (int o = 0; o < 64; o++) {
        float acc = P[kPOffBF1 + o];
        for (int i = 0; i < kPX1; i++)
            acc = fmaf(P[kPOffWF1 + o * kPX1 + i], a[i], acc);
        if (!fused)
            for (int k = 0; k < 5; k++)
                acc = fmaf(P[kPOffWA1 + o * kPXA1 + 64 + k], ang[k], acc);
        b[o] = lrelu(acc);
    }
    layer(kPOffWF2, kPOffBF2, b, 64, a, 64, true, nullptr);                 // spatial feature
    for (int k = 0; k < 5; k++)
        a[64 + k] = fused ? ang[k] : 0.0f;
    layer(kPOffWA1, kPOffBA1, a, kPXA1, b, 64, true, nullptr);             // x (block input)
    layer(kPOffWA2, kPOffBA2, b, 64, a, 64, true, nullptr);
    layer(kPOffWA3, kPOffBA3, a, 64, b, 64, true, b);                      // in place over x
    layer(kPOffWA4, kPOffBA4, b, 64, a, 64, true, nullptr);
    float y[4];
    layer(kPOffWA5, kPOffBA5, a, 64, y, 4, false, nullptr);
    if (out_y4)
        for (int c = 0; c < 4; c++)
            out_y4[c * n + p] = y[c];
    if (out_rgb) {
        // Eq. (8): C = max(y, 0), S = max((e^y - 1) / k, 0), k = 1000 for
        // light from below (transmission), else 100.
        const float k = wi.z < 0.0f ? 10.0f * kSpec : kSpec;
        const DevFabric &fb = fabrics[fid];
        const float C0 = fmaxf(y[0], 0.0f), C1 = fmaxf(y[1], 0.0f);
        const float S0 = fmaxf(expm1f(y[2]) / k, 0.0f), S1 = fmaxf(expm1f(y[3]) / k, 0.0f);
        for (int c = 0; c < 3; c++)
            out_rgb[c * n + p] = fb.kd[0][c] * C0 + fb.kd[1][c] * C1 + fb.ks[0][c] * S0 +
                                 fb.ks[1][c] * S1;
    }
}

template <int P, bool RAW, bool FUSED>
static hipError_t paper_shade(const fabric_gbuffer &g, const DevFabric *fabrics, int n_fabrics,
                              const float *cfold, const void *image, float *out,
                              unsigned long long *err, hipStream_t stream)
{
    using Frag = typename Mfma<P>::Frag;
    const auto *frags = (const Frag *)paper_image_of<P>((void *)image);
    const auto *b5 = (const f32x4 *)(frags + kPFrags * 64);
    const int n_tiles = (int)((g.n + 31) / 32);
    int blocks = (n_tiles + kPaperWaves * kPaperTiles - 1) / (kPaperWaves * kPaperTiles);
    const int cap = device_cus();
    if (blocks > cap)
        blocks = cap;
    const size_t lds = (size_t)kPFrags * 64 * sizeof(Frag) +
                       (size_t)n_fabrics * (64 + kFabCopies * kFabConsts) * sizeof(float);
    hipLaunchKernelGGL((decode_paper_kernel<P, kPaperWaves, kPaperTiles, RAW, FUSED>), dim3(blocks),
                       dim3(64 * kPaperWaves), lds, stream, g, fabrics, n_fabrics, cfold, frags,
                       b5, out, err, n_tiles);
    return hipGetLastError();
}

template <int P>
static hipError_t paper_shade_variant(bool raw, bool fused, const fabric_gbuffer &g,
                                      const DevFabric *fabrics, int n_fabrics, const float *cfold,
                                      const void *image, float *out, unsigned long long *err,
                                      hipStream_t stream)
{
    if (raw)
        return fused ? paper_shade<P, true, true>(g, fabrics, n_fabrics, cfold, image, out, err, stream)
                     : paper_shade<P, true, false>(g, fabrics, n_fabrics, cfold, image, out, err, stream);
    return fused ? paper_shade<P, false, true>(g, fabrics, n_fabrics, cfold, image, out, err, stream)
                 : paper_shade<P, false, false>(g, fabrics, n_fabrics, cfold, image, out, err, stream);
}

hipError_t launch_paper_shade_f32(bool raw, bool fused, const fabric_gbuffer &g,
                                  const DevFabric *fabrics, int n_fabrics, const float *params,
                                  const float *latents, float *out_rgb, float *out_y4,
                                  unsigned long long *err, hipStream_t stream)
{
    if (g.n == 0)
        return hipSuccess;
    const int64_t blocks = (g.n + kRefThreads - 1) / kRefThreads;
    hipLaunchKernelGGL(decode_paper_f32_kernel, dim3((unsigned)blocks), dim3(kRefThreads), 0,
                       stream, g, fabrics, n_fabrics, params, latents, raw ? 1 : 0, fused ? 1 : 0,
                       out_rgb, out_y4, err);
    return hipGetLastError();
}

hipError_t launch_paper_shade(int prec, bool raw, bool fused, const fabric_gbuffer &g,
                              const DevFabric *fabrics, int n_fabrics, const float *cfold,
                              const void *image, float *out, unsigned long long *err,
                              hipStream_t stream)
{
    if (g.n == 0)
        return hipSuccess;
    if (prec == FABRIC_BF16)
        return paper_shade_variant<FABRIC_BF16>(raw, fused, g, fabrics, n_fabrics, cfold, image,
                                                out, err, stream);
    if (prec == FABRIC_FP16)
        return paper_shade_variant<FABRIC_FP16>(raw, fused, g, fabrics, n_fabrics, cfold, image,
                                                out, err, stream);
    return hipErrorInvalidValue;
}

}  // namespace fab
