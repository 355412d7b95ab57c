// Neural shading with an FP8-E4M3 decoder (Sec. 4.2 decoder, Sec. 4.3
// rendering) on the scaled 32x32x64 MFMA: per-layer power-of-two scales,
// FP32 accumulation (see mlp_tile_f8.hpp).
//
// Packing an FP8 decoder takes two launches: a calibration forward in FP32
// over a fixed synthetic batch drawn from the encoded fabrics (one thread
// per sample, plain loops), which records the largest hidden activation of
// each layer, and the packing kernel, which derives the exponents from those
// maxima and from the weights and writes the fragments, the pre-scaled
// biases and the scale header.  The scales thus depend on the parameters and
// the encoded fabrics only, never on the frame being shaded.
#include "mlp_tile_f8.hpp"
#include "shade.hpp"

namespace fab {

namespace {

constexpr int kCalibSamples = 1 << 16;
constexpr int kCalibBlock = 64;
constexpr int kCalibBlocks = kCalibSamples / kCalibBlock;
constexpr uint64_t kCalibSeed = 0x5ca1ab1e0f8ull;

// Image layout: A fragments [NFRAG][64] i32x8, L3's angular BF16 fragments
// [NANG][64] bf16x8, L2 bias [2][64][4] f32x4, L4 bias [64] f32x4, header,
// calibration partial maxima [3][kCalibBlocks].
constexpr size_t kF8FragBytes = (size_t)DecShapeF8::NFRAG * 64 * sizeof(i32x8);
constexpr size_t kF8AngOff = kF8FragBytes;
constexpr size_t kF8Bias2Off = kF8AngOff + (size_t)DecShapeF8::NANG * 64 * sizeof(bf16x8);
constexpr size_t kF8Bias4Off = kF8Bias2Off + (size_t)2 * 64 * 4 * sizeof(f32x4);
constexpr size_t kF8HeaderOff = kF8Bias4Off + (size_t)64 * sizeof(f32x4);
constexpr size_t kF8PartOff = kF8HeaderOff + sizeof(F8Header);
constexpr size_t kF8ImageBytes = kF8PartOff + (size_t)3 * kCalibBlocks * sizeof(float);

// FP32 forward of one calibration sample per thread; per block, the largest
// value of h1, h2, h3 (after ReLU) goes to part[layer][block].
__global__ __launch_bounds__(kCalibBlock) void calib_f8_kernel(
    const float *__restrict__ params, const float *__restrict__ cfold,
    const DevFabric *__restrict__ fabrics, int n_fabrics, float *__restrict__ part)
{
    __shared__ float h[2][kHid][kCalibBlock];
    const int t = threadIdx.x;
    const int q = blockIdx.x * kCalibBlock + t;

    // Sample: fabric uniform over the encoded ones, uv uniform over 8 cells,
    // radius log-uniform over the one-blob encoding's span [2^-14, 4],
    // cosine-distributed directions, a quarter of them lit from below
    // (transmission queries feed wi.z < 0 to the decoder).
    const uint64_t base = 8ull * (uint64_t)q;
    const uint64_t z0 = splitmix64_at(kCalibSeed, base + 0);
    const uint64_t z1 = splitmix64_at(kCalibSeed, base + 1);
    const uint64_t z2 = splitmix64_at(kCalibSeed, base + 2);
    const uint64_t z3 = splitmix64_at(kCalibSeed, base + 3);
    const uint64_t z4 = splitmix64_at(kCalibSeed, base + 4);
    const int fid = (int)((uint32_t)(z0 >> 32) % (uint32_t)n_fabrics);
    const float u = 8.0f * u24_hi(z1), v = 8.0f * u24_mid(z1);
    const float r = exp2f(-14.0f + 16.0f * u24_hi(z2));
    float s, c, xi;
    xi = u24_hi(z3);
    sincospif(2.0f * u24_mid(z3), &s, &c);
    const float wz = sqrtf(1.0f - xi);
    const float3 wi = make_float3(sqrtf(xi) * c, sqrtf(xi) * s,
                                  u24_hi(splitmix64_at(kCalibSeed, base + 5)) < 0.25f ? -wz : wz);
    xi = u24_hi(z4);
    sincospif(2.0f * u24_mid(z4), &s, &c);
    const float3 wo = make_float3(sqrtf(xi) * c, sqrtf(xi) * s, sqrtf(1.0f - xi));

    const DevFabric &f = fabrics[fid];
    float feat[kFeat];
#pragma unroll
    for (int g = 0; g < 2; g++) {
        float s1[kL1Slots32];
        Tile32<FABRIC_BF16>::spatial_slots(u, v, r, f.fwx, f.fwy, f.inv_wx, f.inv_wy, g, s1);
#pragma unroll
        for (int k = 0; k < kL1Slots32; k++)
            feat[l1_feature32(g, k)] = s1[k];
    }

    float m1 = 0.0f, m2 = 0.0f, m3 = 0.0f;
    for (int o = 0; o < kHid; o++) {
        float acc = cfold[fid * kHid + o];
#pragma unroll
        for (int k = 0; k < kFeat; k++)
            acc = fmaf(params[kOffW1 + o * 72 + kLatent + k], feat[k], acc);
        acc = fmaxf(acc, 0.0f);
        m1 = fmaxf(m1, acc);
        h[0][o][t] = acc;
    }
    for (int o = 0; o < kHid; o++) {
        float acc = params[kOffB2 + o];
        for (int k = 0; k < kHid; k++)
            acc = fmaf(params[kOffW2 + o * 64 + k], h[0][k][t], acc);
        acc = fmaxf(acc, 0.0f);
        m2 = fmaxf(m2, acc);
        h[1][o][t] = acc;
    }
    const float x[5] = {wi.x, wi.y, wi.z, wo.x, wo.y};
    for (int o = 0; o < kHid; o++) {
        float acc = params[kOffB3 + o];
        for (int k = 0; k < kHid; k++)
            acc = fmaf(params[kOffW3 + o * 69 + k], h[1][k][t], acc);
#pragma unroll
        for (int a = 0; a < 5; a++)
            acc = fmaf(params[kOffW3 + o * 69 + 64 + a], x[a], acc);
        m3 = fmaxf(m3, fmaxf(acc, 0.0f));
    }
    // Block maxima: a fixed butterfly over the wave (one wave per block).
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        m1 = fmaxf(m1, __shfl_xor(m1, d, 64));
        m2 = fmaxf(m2, __shfl_xor(m2, d, 64));
        m3 = fmaxf(m3, __shfl_xor(m3, d, 64));
    }
    if (t == 0) {
        part[0 * kCalibBlocks + blockIdx.x] = m1;
        part[1 * kCalibBlocks + blockIdx.x] = m2;
        part[2 * kCalibBlocks + blockIdx.x] = m3;
    }
}

// Exponent e with x * 2^e in [2^(top-1), 2^top) for finite x > 0, else 0;
// clamped to +-40 so that every E8M0 scale below stays inside 1..254.
__device__ inline int exp_to(float x, int top)
{
    if (!(x > 0.0f) || !isfinite(x))
        return 0;
    int e;
    frexpf(x, &e);   // x = m 2^e, m in [0.5, 1)
    return min(max(top - e, -40), 40);
}

// Largest |A entry| of layer l (1..4) over the entries the FP8 image holds.
__device__ inline float layer_absmax(const float *__restrict__ params, int layer)
{
    float m = 0.0f;
    if (layer == 1) {
        for (int k = threadIdx.x; k < 64 * kFeat; k += blockDim.x)
            m = fmaxf(m, fabsf(params[kOffW1 + (k / kFeat) * 72 + kLatent + k % kFeat]));
    } else if (layer == 2) {
        for (int k = threadIdx.x; k < 64 * 64; k += blockDim.x)
            m = fmaxf(m, fabsf(params[kOffW2 + k]));
    } else if (layer == 3) {
        // the chained columns only: the angular ones and the bias are BF16
        for (int k = threadIdx.x; k < 64 * 64; k += blockDim.x)
            m = fmaxf(m, fabsf(params[kOffW3 + (k >> 6) * 69 + (k & 63)]));
    } else {
        for (int k = threadIdx.x; k < 4 * 64; k += blockDim.x)
            m = fmaxf(m, fabsf(params[kOffW4 + k]));
    }
    return m;
}

// Block-wide maximum of one value per thread (blockDim.x == 256).
__device__ inline float block_max(float v, float *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if ((int)threadIdx.x < s)
            red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    const float r = red[0];
    __syncthreads();
    return r;
}

// Every block derives the same header from the calibration maxima and the
// weights, then packs its share of the image.
__global__ __launch_bounds__(256) void pack_decoder_f8_kernel(const float *__restrict__ params,
                                                               char *__restrict__ image)
{
    __shared__ float red[256];
    __shared__ F8Header hd;
    const float *part = (const float *)(image + kF8PartOff);
    float hm[3], wm[4];
    for (int l = 0; l < 3; l++) {
        float m = 0.0f;
        for (int b = threadIdx.x; b < kCalibBlocks; b += blockDim.x)
            m = fmaxf(m, part[l * kCalibBlocks + b]);
        hm[l] = block_max(m, red);
    }
    for (int l = 0; l < 4; l++)
        wm[l] = block_max(layer_absmax(params, l + 1), red);
    if (threadIdx.x == 0) {
        int eh[3], ew[4];
        for (int l = 0; l < 3; l++)
            eh[l] = exp_to(hm[l], 7);    // largest activation in [64, 128)
        for (int l = 0; l < 4; l++)
            ew[l] = exp_to(wm[l], 8);    // largest weight in [128, 256)
        const int ein[4] = {kFeatExp, eh[0], eh[1], eh[2]};
        const int eout[4] = {eh[0], eh[1], eh[2], 0};
        for (int l = 0; l < 4; l++) {
            hd.sa[l] = 127 + eout[l] - ew[l];
            hd.sb[l] = 127 - ein[l];
            hd.wmax[l] = wm[l];
            hd.ew[l] = ew[l];
        }
        hd.unused = 0;
        hd.cf_mult = ldexpf(1.0f, eh[0]);
        for (int l = 0; l < 3; l++) {
            hd.hmax[l] = hm[l];
            hd.eh[l] = eh[l];
        }
        for (int k = 0; k < 8; k++)
            hd.pad[k] = 0;
    }
    __syncthreads();

    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < DecShapeF8::NFRAG * 64) {
        const int fr = idx / 64, lane = idx % 64, row = lane & 31, grp = lane >> 5;
        int layer, mb;
        if (fr < DecShapeF8::FRAG_L2) { layer = 1; mb = fr; }
        else if (fr < DecShapeF8::FRAG_L3) { layer = 2; mb = fr - DecShapeF8::FRAG_L2; }
        else if (fr < DecShapeF8::FRAG_L4) { layer = 3; mb = fr - DecShapeF8::FRAG_L3; }
        else { layer = 4; mb = 0; }
        const int m = 32 * mb + row;
        const float sc = ldexpf(1.0f, hd.ew[layer - 1]);
        float w[32];
        for (int j = 0; j < 32; j++) {
            float val = 0.0f;
            if (layer == 1) {
                const int feat = j < kL1Slots32 ? l1_feature32(grp, j) : -1;
                if (feat >= 0) val = params[kOffW1 + m * 72 + kLatent + feat];
            } else if (layer == 2) {
                val = params[kOffW2 + m * 64 + chain32_neuron(grp, j)];
            } else if (layer == 3) {
                val = params[kOffW3 + m * 69 + chain32_neuron(grp, j)];
            } else {
                // 16x16x128 operand: row lane % 16, K block lane / 16
                const int r16 = lane & 15, kb = lane >> 4;
                if (r16 < 4 && (kb & 1) == 0)
                    val = params[kOffW4 + r16 * 64 + chain32_neuron(kb >> 1, j)];
                else if (r16 >= 4 && r16 < 8 && (kb & 1) == 1)
                    val = params[kOffW4 + (r16 - 4) * 64 + chain32_neuron(kb >> 1, j)];
            }
            w[j] = val * sc;
        }
        ((i32x8 *)image)[idx] = pack_f8x32(w);
    }
    if (idx < DecShapeF8::NANG * 64) {
        // L3's angular inputs and bias: BF16 32x32x16 A fragment of M-block
        // mb, lane group g's slots 0..2, weights 2^eh3 W (the FP8 steps'
        // output scale).
        const int mb = idx >> 6, lane = idx & 63, grp = lane >> 5, m = 32 * mb + (lane & 31);
        const float sc = ldexpf(1.0f, hd.eh[2]);
        f32x8 w;
        for (int j = 0; j < 8; j++) {
            const int a = j < 3 ? l3_extra32(grp, j) : -1;
            float val = 0.0f;
            if (a == 5) val = params[kOffB3 + m];
            else if (a >= 0) val = params[kOffW3 + m * 69 + 64 + a];
            w[j] = val * sc;
        }
        ((bf16x8 *)(image + kF8AngOff))[idx] = Mfma<FABRIC_BF16>::from8(w);
    }
    if (idx < 2 * 64 * 4) {
        // bias2[(mb*64 + lane)*4 + q][i] = 2^eh2 b2[row of register 4q + i]
        const int q = idx & 3, lane = (idx >> 2) & 63, mb = idx >> 8, grp = lane >> 5;
        const float sc = ldexpf(1.0f, hd.eh[1]);
        f32x4 b;
        for (int i = 0; i < 4; i++)
            b[i] = params[kOffB2 + 32 * mb + 8 * q + 4 * grp + i] * sc;
        ((f32x4 *)(image + kF8Bias2Off))[idx] = b;
    }
    if (idx < 64) {
        const int grp = idx >> 5;
        f32x4 b;
        for (int i = 0; i < 4; i++)
            b[i] = grp == 0 ? params[kOffB4 + i] : 0.0f;
        ((f32x4 *)(image + kF8Bias4Off))[idx] = b;
    }
    if (idx == 0)
        *(F8Header *)(image + kF8HeaderOff) = hd;
}

template <bool HYBRID>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void decode_f8_kernel(
    fabric_gbuffer g, const DevFabric *__restrict__ fabrics, int n_fabrics,
    const float *__restrict__ cfold, const char *__restrict__ image, FallbackQueue q,
    float *__restrict__ out, unsigned long long *err, int n_tiles)
{
    using FM = FeatureMath<FABRIC_BF16>;
    const F8Header hd = *(const F8Header *)(image + kF8HeaderOff);

    // LDS: L2's C-operand bias by row [64] (register r of lane group g of
    // M-block mb holds row 32 mb + 8 (r / 4) + 4 g + r % 4, so the lanes of a
    // group read the same four rows: broadcast reads), then per fabric
    // 2^eh1 c_f [64], then the staged constants [kFabCopies][n_fabrics][kFabConsts].
    extern __shared__ f32x4 smem4[];
    float *s_b2 = (float *)smem4;
    float *s_cf = s_b2 + 64;
    float *s_fc = s_cf + n_fabrics * 64;
    const f32x4 *bias2 = (const f32x4 *)(image + kF8Bias2Off);   // [2][64 lanes][4]
    for (int k = threadIdx.x; k < 64; k += blockDim.x) {
        const int mb = k >> 5, q4 = (k & 31) >> 3, g = (k & 7) >> 2, i = k & 3;
        s_b2[k] = bias2[(mb * 64 + 32 * g) * 4 + q4][i];
    }
    for (int k = threadIdx.x; k < n_fabrics * 64; k += blockDim.x)
        s_cf[k] = cfold[k] * hd.cf_mult;
    stage_fabric_consts(fabrics, n_fabrics, s_fc);
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int grp = lane >> 5;
    const uint32_t dmask = half_dir_mask(grp);
    const int col = lane & 31;

    i32x8 A[DecShapeF8::NFRAG];
#pragma unroll
    for (int q = 0; q < DecShapeF8::NFRAG; q++)
        A[q] = ((const i32x8 *)image)[q * 64 + lane];
    auto getA = [&](int q) { return A[q]; };
    const f32x4 b4 = ((const f32x4 *)(image + kF8Bias4Off))[lane];
    bf16x8 A3x[DecShapeF8::NANG];
#pragma unroll
    for (int mb = 0; mb < DecShapeF8::NANG; mb++)
        A3x[mb] = ((const bf16x8 *)(image + kF8AngOff))[mb * 64 + lane];

    // The MFMA takes its scales from VGPRs: keep them there for the whole loop.
    F8Header sc = hd;
#pragma unroll
    for (int l = 0; l < 4; l++)
        asm volatile("" : "+v"(sc.sa[l]), "+v"(sc.sb[l]));

    const int n = (int)g.n;
    const int waves = gridDim.x * (blockDim.x >> 6);
    const int wave_id = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const HalfPlanes hp = half_planes(g, grp);
    auto tile_px = [&](int t) { return min((t < n_tiles ? t : wave_id) * 32 + col, n - 1); };

    // Per tile: fault and range decisions, features and the L1 C operand.
    struct Prep {
        int p, fid;     // fid: the staged-constant entry (transmission copy for light from below)
        bool valid, fault, oor;
        i32x8 B1;   // L1's B operand
        bf16x8 x3;  // L3's angular B operand
    };
    auto prepare = [&](const HalfPix &cur, int tile, Prep &r, f32x16 (&a)[2]) {
        r.p = tile * 32 + col;
        r.valid = tile < n_tiles && r.p < n;
        r.fault = pair_any(half_fault(cur, n_fabrics, dmask));
        // Out-of-range rule (r > 1 cell or wo.z < 0.05), decided before the
        // MFMA chain so that no pixel field stays live through it.
        r.oor = HYBRID && !r.fault && pair_any(cur.r > 1.0f || (grp == 1 && cur.xz < 0.05f));
        r.fid = r.fault ? 0 : cur.fid;   // non-finite inputs stay in their own column
        const float *fc = s_fc + r.fid * kFabConsts;
        float s1[kL1Slots32];
        Tile32<FABRIC_BF16>::spatial_slots(cur.uv, cur.uv, cur.r, fc[0], fc[1], fc[2], fc[3], grp,
                                           s1);
        r.B1 = TileF8::l1_operand(s1);
#pragma unroll
        for (int mb = 0; mb < 2; mb++)
#pragma unroll
            for (int q4 = 0; q4 < 4; q4++) {
                const f32x4 c4 = *(const f32x4 *)(s_cf + r.fid * 64 + 32 * mb + 8 * q4 + 4 * grp);
#pragma unroll
                for (int i = 0; i < 4; i++)
                    a[mb][4 * q4 + i] = c4[i];
            }
        // group 1's third slot carries L3's bias
        r.x3 = TileF8::l3x_frag(cur.x0, cur.x1, grp ? 1.0f : cur.xz);
        r.fid = fab_entry(r.fid, n_fabrics, grp ? 1.0f : cur.xz);   // after the c_f reads above
    };
    auto finish = [&](const Prep &r, const f32x16 &y, int tile) {
        // Lanes 0..31 hold y[0..3] of pixel tile*32 + lane.
        if (grp == 0 && r.valid && !r.oor) {
            float rgb[3];
            compose_rgb<FM>(y[0] + b4[0], y[1] + b4[1], y[2] + b4[2], y[3] + b4[3],
                            s_fc + r.fid * kFabConsts, rgb);
#pragma unroll
            for (int c = 0; c < 3; c++)
                plane_store(out, c * n + r.p, r.fault ? 0.0f : rgb[c]);
        }
        const unsigned long long bad = __ballot(grp == 0 && r.valid && r.fault);
        if (lane == 0 && bad)
            atomicAdd(err, (unsigned long long)__popcll(bad));
        if (HYBRID && tile < n_tiles)
            queue_mark32((uint32_t)__ballot(grp == 0 && r.valid && r.oor), tile, q, lane);
    };
    // L2's C operand, read from LDS at each use (holding it would cost 32
    // registers for the whole loop).
    auto getB2 = [&](int mb) {
        f32x16 b;
#pragma unroll
        for (int q4 = 0; q4 < 4; q4++) {
            const f32x4 bq = *(const f32x4 *)(s_b2 + 32 * mb + 8 * q4 + 4 * grp);
#pragma unroll
            for (int i = 0; i < 4; i++)
                b[4 * q4 + i] = bq[i];
        }
        return b;
    };

    // Two tiles per iteration (tile and tile + waves), shaded in alternation;
    // the next pair's fields are loaded while this pair is shaded.
    HalfPix n0 = load_half(g, hp, tile_px(wave_id));
    HalfPix n1 = load_half(g, hp, tile_px(wave_id + waves));
    for (int tile = wave_id; tile < n_tiles; tile += 2 * waves) {
        const HalfPix c0 = n0, c1 = n1;
        n0 = load_half(g, hp, tile_px(tile + 2 * waves));
        n1 = load_half(g, hp, tile_px(tile + 3 * waves));
        Prep r0, r1;
        f32x16 a0[2], a1[2];
        prepare(c0, tile, r0, a0);
        prepare(c1, tile + waves, r1, a1);
        TileF8::forward2(getA, sc, a0, a1, getB2, A3x, r0.B1, r1.B1, r0.x3, r1.x3);
        finish(r0, a0[0], tile);
        finish(r1, a1[0], tile + waves);
    }
}

}  // namespace

size_t f8_image_bytes() { return kF8ImageBytes; }

hipError_t launch_pack_f8(const float *dec_params, const float *cfold, const DevFabric *fabrics,
                          int n_fabrics, void *image, hipStream_t stream)
{
    if (n_fabrics <= 0)
        return hipErrorInvalidValue;
    float *part = (float *)((char *)image + kF8PartOff);
    hipLaunchKernelGGL(calib_f8_kernel, dim3(kCalibBlocks), dim3(kCalibBlock), 0, stream,
                       dec_params, cfold, fabrics, n_fabrics, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const int total = DecShapeF8::NFRAG * 64 > 2 * 64 * 4 ? DecShapeF8::NFRAG * 64 : 2 * 64 * 4;
    hipLaunchKernelGGL(pack_decoder_f8_kernel, dim3((total + 255) / 256), dim3(256), 0, stream,
                       dec_params, (char *)image);
    return hipGetLastError();
}

hipError_t launch_decode_f8(const fabric_gbuffer &g, const DevFabric *fabrics, int n_fabrics,
                            const float *cfold, const void *image, bool hybrid, FallbackQueue q,
                            float *out, unsigned long long *err, hipStream_t stream)
{
    if (g.n == 0)
        return hipSuccess;
    const int n_tiles = (int)((g.n + 31) / 32);
    int blocks = (n_tiles + 3) / 4;
    const int cap = device_cus() * 2;
    if (blocks > cap)
        blocks = cap;
    const size_t lds = (size_t)64 * sizeof(float) +
                       (size_t)n_fabrics * (64 + kFabCopies * kFabConsts) * sizeof(float);
    if (hybrid)
        hipLaunchKernelGGL(decode_f8_kernel<true>, dim3(blocks), dim3(256), lds, stream, g,
                           fabrics, n_fabrics, cfold, (const char *)image, q, out, err, n_tiles);
    else
        hipLaunchKernelGGL(decode_f8_kernel<false>, dim3(blocks), dim3(256), lds, stream, g,
                           fabrics, n_fabrics, cfold, (const char *)image, q, out, err, n_tiles);
    return hipGetLastError();
}

}  // namespace fab
