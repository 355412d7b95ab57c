// C ABI of the fabric library (declared in include/fabric.h): context
// lifetime, argument validation, host-side fabric tables and the launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "kernels.hpp"
#include "paper_train.hpp"
#include "train.hpp"

using namespace fab;

struct fabric_ctx {
    int device = 0;
    float *params = nullptr;          // FP32 masters [decoder | encoder]
    double *adam_m = nullptr;         // FP64 first moments
    double *adam_v = nullptr;         // FP64 second moments
    // Adam step counts on the device, [0] the config network's, [1] the
    // paper-size network's, and their last bias corrections [2][2].
    int64_t *adam_t = nullptr;
    double *adam_corr = nullptr;
    uint64_t weights_version = 1;     // bumped on every parameter change

    int n_mats = 0;
    std::vector<fabric_material> mats;
    DevFabric *fabrics = nullptr;     // [FABRIC_MAX_FABRICS]
    float *enc_inputs = nullptr;      // [FABRIC_MAX_FABRICS][524]
    float *latents = nullptr;         // [FABRIC_MAX_FABRICS][32]
    float *cfold = nullptr;           // [FABRIC_MAX_FABRICS][64]
    LatentLerp *lerp_jobs = nullptr;  // [FABRIC_MAX_FABRICS]
    bool visibility = false;          // V of Eq. (3)-(4) in the analytic filter
    uint64_t table_serial = 0;        // bumped when the fabric table's geometry changes
    uint64_t vis_serial = 0;          // table_serial of the built height texels
    float *vis_tex = nullptr;         // height texels of every fabric
    size_t vis_cap = 0;               // texels allocated
    VisFabric *vis_fab = nullptr;     // [FABRIC_MAX_FABRICS]
    void *paper_image = nullptr;      // paper-size decoder: packed weights
    float *paper_cfold = nullptr;     // [FABRIC_MAX_FABRICS][64]
    int paper_n_mats = 0;             // fabrics folded by the last prepare
    uint64_t paper_serial = 0;        // table_serial of the last prepare
    float *paper_master = nullptr;    // FP32 masters [params | latents [F][64]] or
                                      // [params | encoder] (first prepare)
    bool paper_encoder = false;       // the latents come from the paper-size encoder
    float *paper_latents = nullptr;   // [FABRIC_MAX_FABRICS][64]: the encoder's latents
    double *paper_m = nullptr;        // their FP64 Adam moments
    double *paper_v = nullptr;
    bool paper_raw = false;           // footprint inputs without the one-blob encoding
    bool paper_fused = true;          // false: no spatial fusion stage
    PaperTrainScratch paper_train;
    uint64_t encoded_version = 0;     // weights_version of the last encode
    uint64_t encode_serial = 0;       // bumped on every change of latents or fabric table

    void *image[4] = {nullptr, nullptr, nullptr, nullptr};   // packed decoders
    uint64_t image_version[4] = {0, 0, 0, 0};
    uint64_t image_serial[4] = {0, 0, 0, 0};                 // encode_serial an image was packed for
    void *tmp_image = nullptr;        // packing of caller-supplied parameters
    float *tmp_cfold = nullptr;
    uint16_t *queue_mask = nullptr;   // hybrid frames: pixels routed to the filter
    uint32_t *queue_offsets = nullptr;
    uint32_t *queue_count = nullptr;
    int32_t *queue_idx = nullptr;
    int64_t queue_cap = 0;

    unsigned long long *err = nullptr;
    TrainScratch train;
};

// Fixed device memory of fabric_shade_gbuffer_noalloc: the fallback queue
// (out-of-range mask, scan offsets and block sums, count, pixel indices) of
// frames up to FABRIC_NOALLOC_MAX_PIXELS pixels, 256-byte aligned parts.
// Each GPU the library runs on holds its own copy until the process ends;
// every call on that GPU shares it.
constexpr size_t kNoAllocScratchBytes = (size_t)20 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

// Device address of `scratch` per device (the array's host-side name is not
// a device address), resolved by fabric_create with the device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

hipError_t resolve_scratch(int device)
{
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (device < 0 || device >= kMaxDevices)
        return hipErrorInvalidDevice;
    if (g_scratch_ptr[device])
        return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess)
        return e;
    g_scratch_ptr[device] = p;
    return hipSuccess;
}

void *scratch_of(int device)
{
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    return device >= 0 && device < kMaxDevices ? g_scratch_ptr[device] : nullptr;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// The fallback queue of an n-pixel frame laid out from `base`; returns the
// bytes it spans.
size_t carve_queue(unsigned char *base, int64_t n, FallbackQueue *q)
{
    size_t off = 0;
    q->mask = (uint16_t *)(base + off);
    off = align256(off + (size_t)((n + 31) / 32) * 2 * sizeof(uint16_t));
    q->offsets = (uint32_t *)(base + off);
    off = align256(off + queue_offset_entries(n) * sizeof(uint32_t));
    q->count = (uint32_t *)(base + off);
    off = align256(off + sizeof(uint32_t));
    q->idx = (int32_t *)(base + off);
    off = align256(off + (size_t)n * sizeof(int32_t));
    return off;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess)
            prev = -1;
        if (prev != dev)
            (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (prev >= 0)
            (void)hipSetDevice(prev);
    }
};

hipStream_t as_stream(void *s) { return (hipStream_t)s; }

fabric_status from_hip(hipError_t e)
{
    if (e == hipSuccess)
        return FABRIC_OK;
    if (e == hipErrorOutOfMemory)
        return FABRIC_E_NOMEM;
    return FABRIC_E_DEVICE;
}

template <typename T> fabric_status dalloc(T **p, size_t count)
{
    *p = nullptr;
    if (count == 0)
        return FABRIC_OK;
    return from_hip(hipMalloc((void **)p, count * sizeof(T)));
}

bool finite(float x) { return std::isfinite(x); }

// Validate one fabric; the pattern must hold only 0/1 in its first wx*wy bytes.
bool valid_material(const fabric_material &m)
{
    if (m.wx < 1 || m.wx > FABRIC_MAX_PERIOD || m.wy < 1 || m.wy > FABRIC_MAX_PERIOD)
        return false;
    for (int k = 0; k < m.wx * m.wy; k++)
        if (m.pattern[k] > 1)
            return false;
    for (int y = 0; y < 2; y++) {
        if (!finite(m.alpha[y]) || !(m.alpha[y] > 0.0f) || m.alpha[y] > 1.0f)
            return false;
        if (!finite(m.beta[y]) || m.beta[y] < 0.0f)
            return false;
        if (!finite(m.twist[y]) || !finite(m.incl[y]) || std::fabs(m.incl[y]) > 1.5f)
            return false;
        if (!finite(m.gap[y]) || m.gap[y] < 0.0f || m.gap[y] > 0.9f)
            return false;
        if (!finite(m.wblend[y]) || m.wblend[y] < 0.0f || m.wblend[y] > 1.0f)
            return false;
        for (int c = 0; c < 3; c++)
            if (!finite(m.kd[y][c]) || !finite(m.ks[y][c]))
                return false;
    }
    return true;
}

int top(const fabric_material &m, int i, int j) { return m.pattern[j * m.wx + i]; }

// Per-cell float of the top yarn: run length along the yarn (0 if the yarn
// never goes under) and the cell's offset from the start of its float.
void cell_table(const fabric_material &m, uint16_t cell[256])
{
    std::memset(cell, 0, 256 * sizeof(uint16_t));
    const int wx = m.wx, wy = m.wy;
    for (int j = 0; j < wy; j++) {
        for (int i = 0; i < wx; i++) {
            const int warp = top(m, i, j);
            // Walk along the top yarn: warp floats run over rows of column i,
            // weft floats over columns of row j.
            const int period = warp ? wy : wx;
            auto same = [&](int step) {
                int ii = warp ? i : ((i + step) % wx + wx) % wx;
                int jj = warp ? ((j + step) % wy + wy) % wy : j;
                return top(m, ii, jj) == warp;
            };
            int total = 0;
            for (int s = 0; s < period; s++)
                total += same(s);
            int off = 0, len = 0;
            if (total < period) {
                while (same(-(off + 1)))
                    off++;
                int ahead = 0;
                while (same(ahead + 1))
                    ahead++;
                len = off + ahead + 1;
            }
            cell[j * 16 + i] = (uint16_t)((warp ? 0x8000u : 0u) | ((unsigned)len << 5) | (unsigned)off);
        }
    }
}

DevFabric device_fabric(const fabric_material &m)
{
    DevFabric d;
    std::memset(&d, 0, sizeof(d));
    d.wx = m.wx;
    d.wy = m.wy;
    d.fwx = (float)m.wx;
    d.fwy = (float)m.wy;
    d.inv_wx = (float)(1.0 / m.wx);
    d.inv_wy = (float)(1.0 / m.wy);
    for (int y = 0; y < 2; y++) {
        const double a = m.alpha[y];
        d.alpha[y] = m.alpha[y];
        d.alpha2m1[y] = (float)(1.0 - a * a);
        d.ia2m1[y] = (float)(1.0 / (a * a) - 1.0);
        d.inv_pi_alpha[y] = (float)(1.0 / (M_PI * a));
        d.beta[y] = m.beta[y];
        d.incl[y] = m.incl[y];
        d.cos_twist[y] = (float)std::cos((double)m.twist[y]);
        d.sin_twist[y] = (float)std::sin((double)m.twist[y]);
        const double half = 0.5 * (1.0 - (double)m.gap[y]);
        d.half_width[y] = (float)half;
        d.inv_half_width[y] = (float)(1.0 / half);
        d.wblend[y] = m.wblend[y];
        for (int c = 0; c < 3; c++) {
            d.kd[y][c] = m.kd[y][c];
            d.ks[y][c] = m.ks[y][c];
        }
    }
    cell_table(m, d.cell);
    return d;
}

// Encoder input: per cell (i, j) of a 16x16 grid, [P = 1, P = 0] one-hot inside
// the pattern and zeros outside, then the yarn scalars (warp, weft pairs of
// alpha, beta, twist, inclination, gap, blend) scaled to [0, 1] over fixed
// ranges.
void encoder_input(const fabric_material &m, float x[kEncIn])
{
    std::memset(x, 0, kEncIn * sizeof(float));
    for (int j = 0; j < m.wy; j++)
        for (int i = 0; i < m.wx; i++) {
            const int base = 2 * (16 * j + i);
            x[base + (top(m, i, j) ? 0 : 1)] = 1.0f;
        }
    const double lo[6] = {0.1, 0.0, -M_PI / 6.0, M_PI / 12.0, 0.0, 0.0};
    const double hi[6] = {1.0, 2.0, M_PI / 6.0, M_PI / 4.0, 0.5, 1.0};
    const float *src[6] = {m.alpha, m.beta, m.twist, m.incl, m.gap, m.wblend};
    for (int q = 0; q < 6; q++)
        for (int y = 0; y < 2; y++)
            x[512 + 2 * q + y] = (float)(((double)src[q][y] - lo[q]) / (hi[q] - lo[q]));
}

// Kaiming-uniform weights U(+-sqrt(6/fan_in)), zero biases, from SplitMix64(seed).
void init_params(uint64_t seed, std::vector<float> &out)
{
    out.assign(FABRIC_N_PARAMS, 0.0f);
    struct Layer { int off, outs, ins; };
    const Layer layers[8] = {{kOffW1, 64, 72}, {kOffW2, 64, 64}, {kOffW3, 64, 69}, {kOffW4, 4, 64},
                             {kNDec + kOffE1, 128, 524}, {kNDec + kOffE2, 128, 128},
                             {kNDec + kOffE3, 128, 128}, {kNDec + kOffE4, 32, 128}};
    uint64_t state = seed;
    for (const Layer &L : layers) {
        const double bound = std::sqrt(6.0 / L.ins);
        for (int k = 0; k < L.outs * L.ins; k++) {
            state += 0x9E3779B97F4A7C15ull;
            uint64_t z = state;
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            z ^= z >> 31;
            const double u01 = (double)(z >> 11) * (1.0 / 9007199254740992.0);
            out[L.off + k] = (float)((2.0 * u01 - 1.0) * bound);
        }
    }
}

bool valid_gbuffer(const fabric_gbuffer *g)
{
    // Kernels index pixels with 32-bit integers.
    if (!g || g->n < 0 || g->n > (int64_t)INT32_MAX / 16)
        return false;
    if (g->n == 0)
        return true;
    return g->fabric_id && g->u && g->v && g->radius && g->wi_x && g->wi_y && g->wi_z &&
           g->wo_x && g->wo_y && g->wo_z;
}

bool perfect_square(int n)
{
    if (n <= 0 || n > FABRIC_MAX_SAMPLES)
        return false;
    int s = (int)std::lround(std::sqrt((double)n));
    return s * s == n;
}

// The packed decoder of precision prec for the context's current parameters
// (an FP8 image is calibrated on the encoded fabrics, so it also follows them).
// The images of every precision are allocated by fabric_create; this only
// repacks (a kernel launch, no allocation).
fabric_status ensure_image(fabric_ctx *ctx, int prec, hipStream_t stream)
{
    if (!ctx->image[prec])
        return FABRIC_E_STATE;
    // FP8 scales are calibrated on the encoded fabrics and the BF16 neuron
    // scales bound the activations over their c_f: both follow the encodes.
    const bool fp8 = prec == FABRIC_FP8_E4M3;
    const bool per_encode = fp8 || prec == FABRIC_BF16 || prec == FABRIC_FP16;
    if (ctx->image_version[prec] != ctx->weights_version ||
        (per_encode && ctx->image_serial[prec] != ctx->encode_serial)) {
        fabric_status st =
            fp8 ? from_hip(launch_pack_f8(ctx->params, ctx->cfold, ctx->fabrics, ctx->n_mats,
                                          ctx->image[prec], stream))
                : from_hip(launch_pack_shade(prec, ctx->params, ctx->cfold, ctx->n_mats,
                                             ctx->image[prec], stream));
        if (st != FABRIC_OK)
            return st;
        ctx->image_version[prec] = ctx->weights_version;
        ctx->image_serial[prec] = ctx->encode_serial;
    }
    return FABRIC_OK;
}

// Room for the out-of-range masks, offsets and pixel indices of an n-pixel
// hybrid frame.
// Height of the fabric surface at a point of its period (cells; Eq. (3)-(4)
// visibility).  The slopes that define n_p integrate to
//   across a yarn:    beta half / theta_max  ln cos(theta_max x')
//   along a top float: beta L / (2 incl)     ln cos(incl y')
// with the float's length L in cells; a lower yarn lies one cap depth of the
// cell's top yarn lower (cap: the drop from a yarn's crown to its edge,
// beta half ln(1 / cos theta_max) / theta_max); a hole lies below both caps.
// FP64, each product and quotient taken left to right as written, so that
// the texels rounded to float32 are reproducible.
double surface_height(const fabric_material &m, const uint16_t cell[256], double up, double vp)
{
    const double theta = M_PI / 3.0;
    const int i = std::min((int)std::floor(up), m.wx - 1);
    const int j = std::min((int)std::floor(vp), m.wy - 1);
    const double s = up - i, t = vp - j;
    double half[2], cap[2];
    for (int y = 0; y < 2; y++) {
        half[y] = 0.5 * (1.0 - (double)m.gap[y]);
        cap[y] = (double)m.beta[y] * half[y] * (-std::log(std::cos(theta))) / theta;
    }
    const bool cov_warp = std::fabs(s - 0.5) <= half[0];
    const bool cov_weft = std::fabs(t - 0.5) <= half[1];
    const uint16_t c = cell[j * 16 + i];
    const int top = (c >> 15) ? 0 : 1;   // 0 warp, 1 weft
    int yarn;
    if (top == 0)
        yarn = cov_warp ? 0 : (cov_weft ? 1 : 2);
    else
        yarn = cov_weft ? 1 : (cov_warp ? 0 : 2);
    if (yarn == 2)
        return -cap[top] - cap[1 - top];
    const double across = ((yarn == 0 ? s : t) - 0.5) / half[yarn];
    double h = (double)m.beta[yarn] * half[yarn] / theta * std::log(std::cos(theta * across));
    if (yarn == top) {
        const int len = (c >> 5) & 31, off = c & 31;
        const double incl = (double)m.incl[yarn];
        // A zero inclination leaves the float flat (its limit term is 0).
        if (len > 0 && incl != 0.0) {
            const double along = 2.0 * (off + (yarn == 0 ? t : s)) / len - 1.0;
            h += (double)m.beta[yarn] * (double)len / (2.0 * incl) * std::log(std::cos(incl * along));
        }
    } else {
        h -= cap[top];
    }
    return h;
}

// Height texels of every encoded fabric (kVisRes per cell and axis, the
// height at each texel's centre rounded to float32), uploaded when the
// fabric table changed since the last build.  Returns the arguments of the
// filter launches: V = 1 when visibility is off.
fabric_status ensure_vis(fabric_ctx *ctx, hipStream_t s, VisArgs *out)
{
    *out = VisArgs{nullptr, nullptr};
    if (!ctx->visibility)
        return FABRIC_OK;
    if (ctx->vis_serial != ctx->table_serial || !ctx->vis_tex) {
        std::vector<VisFabric> info(ctx->n_mats);
        size_t total = 0;
        for (int k = 0; k < ctx->n_mats; k++) {
            const fabric_material &m = ctx->mats[k];
            info[k].off = (int32_t)total;
            info[k].tw = m.wx * kVisRes;
            info[k].th = m.wy * kVisRes;
            total += (size_t)info[k].tw * info[k].th;
        }
        std::vector<float> tex(total);
        for (int k = 0; k < ctx->n_mats; k++) {
            const fabric_material &m = ctx->mats[k];
            uint16_t cell[256];
            cell_table(m, cell);
            float hmax = -INFINITY;
            for (int b = 0; b < info[k].th; b++)
                for (int a = 0; a < info[k].tw; a++) {
                    const float h = (float)surface_height(m, cell, (a + 0.5) / kVisRes,
                                                          (b + 0.5) / kVisRes);
                    tex[info[k].off + (size_t)b * info[k].tw + a] = h;
                    hmax = std::max(hmax, h);
                }
            info[k].hmax = hmax;
        }
        if (ctx->vis_cap < total) {
            (void)hipFree(ctx->vis_tex);
            ctx->vis_tex = nullptr;
            ctx->vis_cap = 0;
            fabric_status st = dalloc(&ctx->vis_tex, total);
            if (st != FABRIC_OK)
                return st;
            ctx->vis_cap = total;
        }
        fabric_status st = from_hip(hipMemcpyAsync(ctx->vis_tex, tex.data(), total * sizeof(float),
                                                   hipMemcpyHostToDevice, s));
        if (st == FABRIC_OK)
            st = from_hip(hipMemcpyAsync(ctx->vis_fab, info.data(), info.size() * sizeof(VisFabric),
                                         hipMemcpyHostToDevice, s));
        // The host staging vectors must outlive the copies.
        if (st == FABRIC_OK) st = from_hip(hipStreamSynchronize(s));
        if (st != FABRIC_OK)
            return st;
        ctx->vis_serial = ctx->table_serial;
    }
    *out = VisArgs{ctx->vis_tex, ctx->vis_fab};
    return FABRIC_OK;
}

fabric_status ensure_queue(fabric_ctx *ctx, int64_t n)
{
    if (!ctx->queue_count) {
        fabric_status st = dalloc(&ctx->queue_count, 1);
        if (st != FABRIC_OK)
            return st;
    }
    if (ctx->queue_cap >= n)
        return FABRIC_OK;
    (void)hipFree(ctx->queue_mask);
    (void)hipFree(ctx->queue_offsets);
    (void)hipFree(ctx->queue_idx);
    ctx->queue_mask = nullptr;
    ctx->queue_offsets = nullptr;
    ctx->queue_idx = nullptr;
    ctx->queue_cap = 0;
    fabric_status st = dalloc(&ctx->queue_mask, (size_t)((n + 31) / 32) * 2);
    if (st == FABRIC_OK)
        st = dalloc(&ctx->queue_offsets, queue_offset_entries(n));
    if (st == FABRIC_OK)
        st = dalloc(&ctx->queue_idx, (size_t)n);
    if (st == FABRIC_OK)
        ctx->queue_cap = n;
    return st;
}

// The paper-size network's latents: the masters' own (latents trained as
// parameters) or those the encoder last produced.
const float *paper_latents_of(const fabric_ctx *ctx)
{
    return ctx->paper_encoder ? ctx->paper_latents
                              : ctx->paper_master + FABRIC_N_PAPER_DECODER_PARAMS;
}

// Masters and Adam moments of the paper-size network, sized for either layout.
constexpr size_t kPaperMasterFloats =
    (size_t)FABRIC_N_PAPER_DECODER_PARAMS +
    ((size_t)FABRIC_MAX_FABRICS * FABRIC_PAPER_LATENT > (size_t)FABRIC_N_PAPER_ENCODER_PARAMS
         ? (size_t)FABRIC_MAX_FABRICS * FABRIC_PAPER_LATENT
         : (size_t)FABRIC_N_PAPER_ENCODER_PARAMS);

fabric_status ensure_paper_master(fabric_ctx *ctx)
{
    if (ctx->paper_master)
        return FABRIC_OK;
    fabric_status st = dalloc(&ctx->paper_master, kPaperMasterFloats);
    if (st == FABRIC_OK) st = dalloc(&ctx->paper_m, kPaperMasterFloats);
    if (st == FABRIC_OK) st = dalloc(&ctx->paper_v, kPaperMasterFloats);
    if (st == FABRIC_OK) st = dalloc(&ctx->paper_latents, (size_t)FABRIC_MAX_FABRICS * FABRIC_PAPER_LATENT);
    if (st != FABRIC_OK) {
        (void)hipFree(ctx->paper_master);
        (void)hipFree(ctx->paper_m);
        (void)hipFree(ctx->paper_v);
        (void)hipFree(ctx->paper_latents);
        ctx->paper_master = ctx->paper_latents = nullptr;
        ctx->paper_m = ctx->paper_v = nullptr;
    }
    return st;
}

bool supported_prec(int prec)
{
    return prec == FABRIC_FP32 || prec == FABRIC_BF16 || prec == FABRIC_FP16 || prec == FABRIC_FP8_E4M3;
}

}  // namespace

extern "C" {

const char *fabric_status_str(fabric_status s)
{
    switch (s) {
    case FABRIC_OK: return "ok";
    case FABRIC_E_INVAL: return "invalid argument";
    case FABRIC_E_RANGE: return "out of range";
    case FABRIC_E_NOMEM: return "out of device memory";
    case FABRIC_E_DEVICE: return "HIP runtime error";
    case FABRIC_E_NONFINITE: return "non-finite loss";
    case FABRIC_E_STATE: return "invalid call order";
    }
    return "unknown status";
}

void fabric_destroy(fabric_ctx *ctx)
{
    if (!ctx)
        return;
    DeviceGuard guard(ctx->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(ctx->params);
    (void)hipFree(ctx->adam_m);
    (void)hipFree(ctx->adam_v);
    (void)hipFree(ctx->adam_t);
    (void)hipFree(ctx->adam_corr);
    (void)hipFree(ctx->fabrics);
    (void)hipFree(ctx->enc_inputs);
    (void)hipFree(ctx->latents);
    (void)hipFree(ctx->cfold);
    (void)hipFree(ctx->lerp_jobs);
    (void)hipFree(ctx->vis_tex);
    (void)hipFree(ctx->vis_fab);
    (void)hipFree(ctx->paper_image);
    (void)hipFree(ctx->paper_cfold);
    (void)hipFree(ctx->paper_master);
    (void)hipFree(ctx->paper_m);
    (void)hipFree(ctx->paper_v);
    (void)hipFree(ctx->paper_latents);
    paper_train_scratch_free(ctx->paper_train);
    for (int k = 0; k < 4; k++)
        (void)hipFree(ctx->image[k]);
    (void)hipFree(ctx->tmp_image);
    (void)hipFree(ctx->queue_mask);
    (void)hipFree(ctx->queue_offsets);
    (void)hipFree(ctx->queue_count);
    (void)hipFree(ctx->queue_idx);
    (void)hipFree(ctx->tmp_cfold);
    (void)hipFree(ctx->err);
    train_scratch_free(ctx->train);
    delete ctx;
}

fabric_status fabric_create(fabric_ctx **out, int device, uint64_t seed)
{
    if (!out)
        return FABRIC_E_INVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
        return FABRIC_E_DEVICE;
    if (device < 0 || device >= count)
        return FABRIC_E_INVAL;
    fabric_ctx *ctx = new (std::nothrow) fabric_ctx();
    if (!ctx)
        return FABRIC_E_NOMEM;
    ctx->device = device;
    DeviceGuard guard(device);
    fabric_status st = FABRIC_OK;
    const size_t F = FABRIC_MAX_FABRICS;
    if (st == FABRIC_OK) st = dalloc(&ctx->params, FABRIC_N_PARAMS);
    if (st == FABRIC_OK) st = dalloc(&ctx->adam_m, FABRIC_N_PARAMS);
    if (st == FABRIC_OK) st = dalloc(&ctx->adam_v, FABRIC_N_PARAMS);
    if (st == FABRIC_OK) st = dalloc(&ctx->adam_t, 2);
    if (st == FABRIC_OK) st = dalloc(&ctx->adam_corr, 4);
    if (st == FABRIC_OK) st = dalloc(&ctx->fabrics, F);
    if (st == FABRIC_OK) st = dalloc(&ctx->enc_inputs, F * kEncIn);
    if (st == FABRIC_OK) st = dalloc(&ctx->latents, F * kLatent);
    if (st == FABRIC_OK) st = dalloc(&ctx->cfold, F * 64);
    if (st == FABRIC_OK) st = dalloc(&ctx->tmp_cfold, F * 64);
    if (st == FABRIC_OK) st = dalloc(&ctx->lerp_jobs, F);
    if (st == FABRIC_OK) st = dalloc(&ctx->vis_fab, F);
    if (st == FABRIC_OK) st = dalloc((char **)&ctx->paper_image, paper_image_bytes());
    if (st == FABRIC_OK) st = dalloc(&ctx->paper_cfold, F * 64);
    if (st == FABRIC_OK) st = dalloc(&ctx->err, 1);
    if (st == FABRIC_OK) {
        const size_t img = decoder_image_bytes(FABRIC_FP32);   // the largest image
        st = from_hip(hipMalloc(&ctx->tmp_image, img));
    }
    for (int prec = 0; prec < 4 && st == FABRIC_OK; prec++)
        st = from_hip(hipMalloc(&ctx->image[prec], shade_image_bytes(prec)));
    if (st == FABRIC_OK) st = from_hip(resolve_scratch(device));
    if (st == FABRIC_OK) {
        std::vector<float> p;
        init_params(seed, p);
        st = from_hip(hipMemcpy(ctx->params, p.data(), p.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    if (st == FABRIC_OK) st = from_hip(hipMemset(ctx->adam_m, 0, FABRIC_N_PARAMS * sizeof(double)));
    if (st == FABRIC_OK) st = from_hip(hipMemset(ctx->adam_v, 0, FABRIC_N_PARAMS * sizeof(double)));
    if (st == FABRIC_OK) st = from_hip(hipMemset(ctx->adam_t, 0, 2 * sizeof(int64_t)));
    if (st == FABRIC_OK) st = from_hip(hipMemset(ctx->adam_corr, 0, 4 * sizeof(double)));
    if (st == FABRIC_OK) st = from_hip(hipMemset(ctx->err, 0, sizeof(unsigned long long)));
    if (st == FABRIC_OK) st = from_hip(hipDeviceSynchronize());
    if (st != FABRIC_OK) {
        fabric_destroy(ctx);
        return st;
    }
    *out = ctx;
    return FABRIC_OK;
}

fabric_status fabric_encode(fabric_ctx *ctx, const fabric_material *mats, int32_t n_mats, void *stream)
{
    if (!ctx || !mats)
        return FABRIC_E_INVAL;
    if (n_mats < 1 || n_mats > FABRIC_MAX_FABRICS)
        return FABRIC_E_RANGE;
    for (int k = 0; k < n_mats; k++)
        if (!valid_material(mats[k]))
            return FABRIC_E_INVAL;
    DeviceGuard guard(ctx->device);
    hipStream_t s = as_stream(stream);
    std::vector<DevFabric> dev(n_mats);
    std::vector<float> inputs((size_t)n_mats * kEncIn);
    for (int k = 0; k < n_mats; k++) {
        dev[k] = device_fabric(mats[k]);
        encoder_input(mats[k], inputs.data() + (size_t)k * kEncIn);
    }
    fabric_status st = from_hip(hipMemcpyAsync(ctx->fabrics, dev.data(), dev.size() * sizeof(DevFabric),
                                               hipMemcpyHostToDevice, s));
    if (st == FABRIC_OK)
        st = from_hip(hipMemcpyAsync(ctx->enc_inputs, inputs.data(), inputs.size() * sizeof(float),
                                     hipMemcpyHostToDevice, s));
    // The host staging vectors must outlive the copies.
    if (st == FABRIC_OK) st = from_hip(hipStreamSynchronize(s));
    if (st == FABRIC_OK)
        st = from_hip(launch_encoder_forward(ctx->params + kNDec, ctx->enc_inputs, n_mats, ctx->latents, s));
    if (st == FABRIC_OK)
        st = from_hip(launch_fold_latents(ctx->params, ctx->latents, n_mats, ctx->cfold, s));
    if (st != FABRIC_OK)
        return st;
    ctx->mats.assign(mats, mats + n_mats);
    ctx->n_mats = n_mats;
    ctx->encoded_version = ctx->weights_version;
    ctx->encode_serial += 1;
    ctx->table_serial += 1;
    return FABRIC_OK;
}

fabric_status fabric_set_albedo(fabric_ctx *ctx, int32_t fabric, const float kd[2][3],
                                const float ks[2][3], void *stream)
{
    if (!ctx || !kd || !ks)
        return FABRIC_E_INVAL;
    if (ctx->n_mats == 0)
        return FABRIC_E_STATE;
    if (fabric < 0 || fabric >= ctx->n_mats)
        return FABRIC_E_RANGE;
    for (int y = 0; y < 2; y++)
        for (int c = 0; c < 3; c++)
            if (!finite(kd[y][c]) || !finite(ks[y][c]))
                return FABRIC_E_INVAL;
    DeviceGuard guard(ctx->device);
    fabric_material &m = ctx->mats[fabric];
    std::memcpy(m.kd, kd, sizeof(m.kd));
    std::memcpy(m.ks, ks, sizeof(m.ks));
    DevFabric d = device_fabric(m);
    hipStream_t s = as_stream(stream);
    fabric_status st = from_hip(hipMemcpyAsync(ctx->fabrics + fabric, &d, sizeof(DevFabric),
                                               hipMemcpyHostToDevice, s));
    if (st == FABRIC_OK)
        st = from_hip(hipStreamSynchronize(s));
    return st;
}

fabric_status fabric_paper_prepare(fabric_ctx *ctx, const float *params, const float *latents,
                                   void *stream)
{
    if (!ctx || !params || !latents)
        return FABRIC_E_INVAL;
    if (ctx->n_mats == 0)
        return FABRIC_E_STATE;
    DeviceGuard guard(ctx->device);
    const size_t total = kPaperMasterFloats;
    fabric_status st = ensure_paper_master(ctx);
    if (st != FABRIC_OK)
        return st;
    ctx->paper_encoder = false;
    // The context keeps its own copy (the masters training updates).
    hipStream_t s = as_stream(stream);
    float *pm = ctx->paper_master, *lm = ctx->paper_master + FABRIC_N_PAPER_DECODER_PARAMS;
    st = from_hip(hipMemcpyAsync(pm, params, FABRIC_N_PAPER_DECODER_PARAMS * sizeof(float),
                                 hipMemcpyDeviceToDevice, s));
    if (st == FABRIC_OK)
        st = from_hip(hipMemcpyAsync(lm, latents, (size_t)ctx->n_mats * FABRIC_PAPER_LATENT * sizeof(float),
                                     hipMemcpyDeviceToDevice, s));
    if (st == FABRIC_OK) st = from_hip(hipMemsetAsync(ctx->paper_m, 0, total * sizeof(double), s));
    if (st == FABRIC_OK) st = from_hip(hipMemsetAsync(ctx->paper_v, 0, total * sizeof(double), s));
    if (st == FABRIC_OK) st = from_hip(hipMemsetAsync(ctx->adam_t + 1, 0, sizeof(int64_t), s));
    if (st == FABRIC_OK)
        st = from_hip(launch_paper_prepare(pm, lm, ctx->n_mats, ctx->paper_fused, ctx->paper_image,
                                           ctx->paper_cfold, s));
    if (st != FABRIC_OK) {
        ctx->paper_n_mats = 0;
        return st;
    }
    ctx->paper_n_mats = ctx->n_mats;
    ctx->paper_serial = ctx->table_serial;
    return FABRIC_OK;
}

fabric_status fabric_paper_prepare_encoder(fabric_ctx *ctx, const float *params,
                                           const float *enc_params, void *stream)
{
    if (!ctx || !params || !enc_params)
        return FABRIC_E_INVAL;
    if (ctx->n_mats == 0)
        return FABRIC_E_STATE;
    DeviceGuard guard(ctx->device);
    fabric_status st = ensure_paper_master(ctx);
    if (st != FABRIC_OK)
        return st;
    hipStream_t s = as_stream(stream);
    float *pm = ctx->paper_master, *em = ctx->paper_master + FABRIC_N_PAPER_DECODER_PARAMS;
    st = from_hip(hipMemcpyAsync(pm, params, FABRIC_N_PAPER_DECODER_PARAMS * sizeof(float),
                                 hipMemcpyDeviceToDevice, s));
    if (st == FABRIC_OK)
        st = from_hip(hipMemcpyAsync(em, enc_params, FABRIC_N_PAPER_ENCODER_PARAMS * sizeof(float),
                                     hipMemcpyDeviceToDevice, s));
    if (st == FABRIC_OK) st = from_hip(hipMemsetAsync(ctx->paper_m, 0, kPaperMasterFloats * sizeof(double), s));
    if (st == FABRIC_OK) st = from_hip(hipMemsetAsync(ctx->paper_v, 0, kPaperMasterFloats * sizeof(double), s));
    if (st == FABRIC_OK) st = from_hip(hipMemsetAsync(ctx->adam_t + 1, 0, sizeof(int64_t), s));
    ctx->paper_encoder = true;
    ctx->paper_n_mats = 0;
    if (st != FABRIC_OK)
        return st;
    return fabric_paper_encode(ctx, stream);
}

fabric_status fabric_paper_encode(fabric_ctx *ctx, void *stream)
{
    if (!ctx)
        return FABRIC_E_INVAL;
    if (ctx->n_mats == 0 || !ctx->paper_master || !ctx->paper_encoder)
        return FABRIC_E_STATE;
    DeviceGuard guard(ctx->device);
    hipStream_t s = as_stream(stream);
    hipError_t e = launch_encoder_forward_n(ctx->paper_master + FABRIC_N_PAPER_DECODER_PARAMS,
                                            ctx->enc_inputs, ctx->n_mats, FABRIC_PAPER_LATENT,
                                            ctx->paper_latents, s);
    if (e == hipSuccess)
        e = launch_paper_prepare(ctx->paper_master, ctx->paper_latents, ctx->n_mats,
                                 ctx->paper_fused, ctx->paper_image, ctx->paper_cfold, s);
    if (e != hipSuccess) {
        ctx->paper_n_mats = 0;
        return from_hip(e);
    }
    ctx->paper_n_mats = ctx->n_mats;
    ctx->paper_serial = ctx->table_serial;
    return FABRIC_OK;
}

fabric_status fabric_paper_get_encoder(fabric_ctx *ctx, float *enc_params_host)
{
    if (!ctx || !enc_params_host)
        return FABRIC_E_INVAL;
    if (!ctx->paper_master || !ctx->paper_encoder)
        return FABRIC_E_STATE;
    DeviceGuard guard(ctx->device);
    fabric_status st = from_hip(hipDeviceSynchronize());
    if (st == FABRIC_OK)
        st = from_hip(hipMemcpy(enc_params_host, ctx->paper_master + FABRIC_N_PAPER_DECODER_PARAMS,
                                FABRIC_N_PAPER_ENCODER_PARAMS * sizeof(float),
                                hipMemcpyDeviceToHost));
    return st;
}

fabric_status fabric_paper_shade(fabric_ctx *ctx, const fabric_gbuffer *g, fabric_prec prec,
                                 float *out_rgb, void *stream)
{
    if (!ctx || !valid_gbuffer(g) || (g->n > 0 && !out_rgb))
        return FABRIC_E_INVAL;
    if (prec != FABRIC_BF16 && prec != FABRIC_FP16 && prec != FABRIC_FP32)
        return FABRIC_E_INVAL;
    if (ctx->paper_n_mats == 0 || ctx->paper_serial != ctx->table_serial)
        return FABRIC_E_STATE;
    if (g->n == 0)
        return FABRIC_OK;
    DeviceGuard guard(ctx->device);
    if (prec == FABRIC_FP32)
        return from_hip(launch_paper_shade_f32(
            ctx->paper_raw, ctx->paper_fused, *g, ctx->fabrics, ctx->paper_n_mats,
            ctx->paper_master, paper_latents_of(ctx), out_rgb, nullptr, ctx->err,
            as_stream(stream)));
    return from_hip(launch_paper_shade(prec, ctx->paper_raw, ctx->paper_fused, *g, ctx->fabrics, ctx->n_mats, ctx->paper_cfold,
                                       ctx->paper_image, out_rgb, ctx->err, as_stream(stream)));
}

fabric_status fabric_paper_forward(fabric_ctx *ctx, const fabric_gbuffer *g, float *y4,
                                   void *stream)
{
    if (!ctx || !valid_gbuffer(g) || (g->n > 0 && !y4))
        return FABRIC_E_INVAL;
    if (ctx->paper_n_mats == 0 || ctx->paper_serial != ctx->table_serial)
        return FABRIC_E_STATE;
    if (g->n == 0)
        return FABRIC_OK;
    DeviceGuard guard(ctx->device);
    return from_hip(launch_paper_shade_f32(
        ctx->paper_raw, ctx->paper_fused, *g, ctx->fabrics, ctx->paper_n_mats, ctx->paper_master,
        paper_latents_of(ctx), nullptr, y4, ctx->err, as_stream(stream)));
}

fabric_status fabric_set_visibility(fabric_ctx *ctx, int32_t enable)
{
    if (!ctx || (enable != 0 && enable != 1))
        return FABRIC_E_INVAL;
    ctx->visibility = enable != 0;
    return FABRIC_OK;
}

fabric_status fabric_lerp_latents(fabric_ctx *ctx, const int32_t *dst, const int32_t *a,
                                  const int32_t *b, const float *t, int32_t count, void *stream)
{
    if (!ctx)
        return FABRIC_E_INVAL;
    if (ctx->n_mats == 0 || ctx->encoded_version != ctx->weights_version)
        return FABRIC_E_STATE;
    if (count < 0 || count > ctx->n_mats)
        return FABRIC_E_RANGE;
    if (count == 0)
        return FABRIC_OK;
    if (!dst || !a || !b || !t)
        return FABRIC_E_INVAL;
    std::vector<LatentLerp> jobs(count);
    std::vector<char> taken(ctx->n_mats, 0);
    for (int k = 0; k < count; k++) {
        const int32_t idx[3] = {dst[k], a[k], b[k]};
        for (int32_t i : idx)
            if (i < 0 || i >= ctx->n_mats)
                return FABRIC_E_RANGE;
        if (!finite(t[k]) || taken[dst[k]])
            return FABRIC_E_INVAL;
        taken[dst[k]] = 1;
        jobs[k] = LatentLerp{dst[k], a[k], b[k], t[k]};
    }
    DeviceGuard guard(ctx->device);
    hipStream_t s = as_stream(stream);
    fabric_status st = from_hip(hipMemcpyAsync(ctx->lerp_jobs, jobs.data(),
                                               jobs.size() * sizeof(LatentLerp),
                                               hipMemcpyHostToDevice, s));
    // The host staging vector must outlive the copy.
    if (st == FABRIC_OK) st = from_hip(hipStreamSynchronize(s));
    if (st == FABRIC_OK) st = from_hip(launch_lerp_latents(ctx->lerp_jobs, count, ctx->latents, s));
    if (st == FABRIC_OK)
        st = from_hip(launch_fold_latents(ctx->params, ctx->latents, ctx->n_mats, ctx->cfold, s));
    // Even a failed launch may have changed latents: force FP8 recalibration.
    ctx->encode_serial += 1;
    return st;
}

fabric_status fabric_shade_gbuffer(fabric_ctx *ctx, const fabric_gbuffer *g, fabric_prec prec,
                                   int32_t fallback_samples, uint64_t seed, float *out_rgb,
                                   void *stream)
{
    if (!ctx || !valid_gbuffer(g) || (g->n > 0 && !out_rgb))
        return FABRIC_E_INVAL;
    if (!supported_prec(prec))
        return FABRIC_E_INVAL;
    if (fallback_samples < 0 || (fallback_samples > 0 && !perfect_square(fallback_samples)))
        return FABRIC_E_INVAL;
    if (ctx->n_mats == 0 || ctx->encoded_version != ctx->weights_version)
        return FABRIC_E_STATE;
    if (g->n == 0)
        return FABRIC_OK;
    DeviceGuard guard(ctx->device);
    hipStream_t s = as_stream(stream);
    fabric_status st = ensure_image(ctx, prec, s);
    VisArgs vis{nullptr, nullptr};
    if (st == FABRIC_OK && fallback_samples > 0)
        st = ensure_queue(ctx, g->n);
    if (st == FABRIC_OK && fallback_samples > 0)
        st = ensure_vis(ctx, s, &vis);
    if (st != FABRIC_OK)
        return st;
    const FallbackQueue q{ctx->queue_mask, ctx->queue_offsets, ctx->queue_count, ctx->queue_idx};
    return from_hip(launch_decode(prec, false, *g, ctx->fabrics, ctx->n_mats, ctx->cfold,
                                  ctx->image[prec], fallback_samples, seed, vis, q, out_rgb,
                                  ctx->err, s));
}

fabric_status fabric_shade_gbuffer_noalloc(fabric_ctx *ctx, const fabric_gbuffer *g,
                                           fabric_prec prec, int32_t fallback_samples,
                                           uint64_t seed, float *out_rgb, void *stream)
{
    if (!ctx || !valid_gbuffer(g) || (g->n > 0 && !out_rgb))
        return FABRIC_E_INVAL;
    if (!supported_prec(prec))
        return FABRIC_E_INVAL;
    if (fallback_samples < 0 || (fallback_samples > 0 && !perfect_square(fallback_samples)))
        return FABRIC_E_INVAL;
    if (g->n > FABRIC_NOALLOC_MAX_PIXELS)
        return FABRIC_E_RANGE;
    if (ctx->n_mats == 0 || ctx->encoded_version != ctx->weights_version)
        return FABRIC_E_STATE;
    // The height texels are built (and allocated) by the other entry points.
    if (fallback_samples > 0 && ctx->visibility &&
        (!ctx->vis_tex || ctx->vis_serial != ctx->table_serial))
        return FABRIC_E_STATE;
    if (g->n == 0)
        return FABRIC_OK;
    unsigned char *base = (unsigned char *)scratch_of(ctx->device);
    if (!base)
        return FABRIC_E_STATE;
    FallbackQueue q{nullptr, nullptr, nullptr, nullptr};
    if (carve_queue(base, g->n, &q) > kNoAllocScratchBytes)
        return FABRIC_E_RANGE;
    DeviceGuard guard(ctx->device);
    hipStream_t s = as_stream(stream);
    fabric_status st = ensure_image(ctx, prec, s);
    if (st != FABRIC_OK)
        return st;
    VisArgs vis{nullptr, nullptr};
    if (fallback_samples > 0 && ctx->visibility)
        vis = VisArgs{ctx->vis_tex, ctx->vis_fab};
    return from_hip(launch_decode(prec, false, *g, ctx->fabrics, ctx->n_mats, ctx->cfold,
                                  ctx->image[prec], fallback_samples, seed, vis, q, out_rgb,
                                  ctx->err, s));
}

fabric_status fabric_gt_filtered(fabric_ctx *ctx, const fabric_gbuffer *g, int32_t n_samples,
                                 uint64_t seed, float *out_rgb, float *out_comp, void *stream)
{
    if (!ctx || !valid_gbuffer(g) || (!out_rgb && !out_comp) || !perfect_square(n_samples))
        return FABRIC_E_INVAL;
    if (ctx->n_mats == 0)
        return FABRIC_E_STATE;
    if (g->n == 0)
        return FABRIC_OK;
    DeviceGuard guard(ctx->device);
    hipStream_t s = as_stream(stream);
    VisArgs vis;
    fabric_status st = ensure_vis(ctx, s, &vis);
    if (st != FABRIC_OK)
        return st;
    return from_hip(launch_gt_filter(*g, ctx->fabrics, ctx->n_mats, n_samples, seed, vis, out_rgb,
                                     out_comp, ctx->err, s));
}

fabric_status fabric_decoder_forward(fabric_ctx *ctx, const fabric_gbuffer *g, fabric_prec prec,
                                     const float *dec_params, const float *latents, float *y4,
                                     void *stream)
{
    if (!ctx || !valid_gbuffer(g) || !dec_params || !latents || (g->n > 0 && !y4))
        return FABRIC_E_INVAL;
    if (prec != FABRIC_FP32 && prec != FABRIC_BF16)
        return FABRIC_E_INVAL;
    if (ctx->n_mats == 0)
        return FABRIC_E_STATE;
    if (g->n == 0)
        return FABRIC_OK;
    DeviceGuard guard(ctx->device);
    hipStream_t s = as_stream(stream);
    fabric_status st = from_hip(launch_pack_decoder(prec, dec_params, ctx->tmp_image, s));
    if (st == FABRIC_OK)
        st = from_hip(launch_fold_latents(dec_params, latents, ctx->n_mats, ctx->tmp_cfold, s));
    if (st == FABRIC_OK)
        st = from_hip(launch_decode(prec, true, *g, ctx->fabrics, ctx->n_mats, ctx->tmp_cfold,
                                    ctx->tmp_image, 0, 0, VisArgs{nullptr, nullptr},
                                    FallbackQueue{nullptr, nullptr, nullptr, nullptr}, y4,
                                    ctx->err, s));
    // The next shade must repack: tmp buffers are separate, so nothing else is stale.
    return st;
}

fabric_status fabric_decoder_backward(fabric_ctx *ctx, const fabric_gbuffer *g,
                                      const float *dec_params, const float *latents,
                                      const float *grad_y4, float *grad_params,
                                      float *grad_latents, void *stream)
{
    if (!ctx || !valid_gbuffer(g) || !dec_params || !latents || !grad_params || !grad_latents ||
        (g->n > 0 && !grad_y4))
        return FABRIC_E_INVAL;
    if (ctx->n_mats == 0)
        return FABRIC_E_STATE;
    DeviceGuard guard(ctx->device);
    return from_hip(decoder_backward(ctx->train, *g, ctx->fabrics, ctx->n_mats, dec_params, latents,
                                     grad_y4, grad_params, grad_latents, as_stream(stream)));
}

fabric_status fabric_encoder_forward(fabric_ctx *ctx, const float *enc_params, float *latents,
                                     void *stream)
{
    if (!ctx || !enc_params || !latents)
        return FABRIC_E_INVAL;
    if (ctx->n_mats == 0)
        return FABRIC_E_STATE;
    DeviceGuard guard(ctx->device);
    return from_hip(launch_encoder_forward(enc_params, ctx->enc_inputs, ctx->n_mats, latents,
                                           as_stream(stream)));
}

fabric_status fabric_encoder_backward(fabric_ctx *ctx, const float *enc_params,
                                      const float *grad_latents, float *grad_enc_params,
                                      void *stream)
{
    if (!ctx || !enc_params || !grad_latents || !grad_enc_params)
        return FABRIC_E_INVAL;
    if (ctx->n_mats == 0)
        return FABRIC_E_STATE;
    DeviceGuard guard(ctx->device);
    return from_hip(encoder_backward(ctx->train, enc_params, ctx->enc_inputs, ctx->n_mats,
                                     grad_latents, grad_enc_params, as_stream(stream)));
}

fabric_status fabric_make_batch(fabric_ctx *ctx, uint64_t seed, int64_t n, float r_lo, float r_hi,
                                float btdf_frac, const fabric_gbuffer_out *out, void *stream)
{
    if (!ctx || !out || n < 0 || out->n < n || !(r_lo > 0.0f) || !(r_hi >= r_lo) || !finite(r_hi))
        return FABRIC_E_INVAL;
    if (!(btdf_frac >= 0.0f && btdf_frac <= 1.0f))
        return FABRIC_E_INVAL;
    if (n > 0 && !(out->fabric_id && out->u && out->v && out->radius && out->wi_x && out->wi_y &&
                   out->wi_z && out->wo_x && out->wo_y && out->wo_z))
        return FABRIC_E_INVAL;
    if (ctx->n_mats == 0)
        return FABRIC_E_STATE;
    if (n == 0)
        return FABRIC_OK;
    DeviceGuard guard(ctx->device);
    return from_hip(launch_make_batch(seed, n, ctx->n_mats, r_lo, r_hi, btdf_frac, *out,
                                      as_stream(stream)));
}

namespace {
fabric_status check_train_args(fabric_ctx *ctx, const fabric_gbuffer *batch, const float *targets,
                               const fabric_train_cfg *cfg)
{
    if (!ctx || !cfg)
        return FABRIC_E_INVAL;
    if (batch && !valid_gbuffer(batch))
        return FABRIC_E_INVAL;
    if (targets && !batch)
        return FABRIC_E_INVAL;
    if (!batch && (cfg->batch < 1 || cfg->batch > ((int64_t)1 << 26)))
        return FABRIC_E_RANGE;
    if (!targets && !perfect_square(cfg->gt_samples))
        return FABRIC_E_INVAL;
    if (cfg->prec != FABRIC_FP32 && cfg->prec != FABRIC_BF16)
        return FABRIC_E_INVAL;
    if (!batch && !(cfg->btdf_frac >= 0.0f && cfg->btdf_frac <= 1.0f))
        return FABRIC_E_INVAL;
    if (!std::isfinite(cfg->lr) || cfg->lr < 0.0 || !(cfg->beta1 >= 0.0 && cfg->beta1 < 1.0) ||
        !(cfg->beta2 >= 0.0 && cfg->beta2 < 1.0) || !(cfg->eps > 0.0))
        return FABRIC_E_INVAL;
    if (!batch && (!(cfg->r_lo > 0.0f) || !(cfg->r_hi >= cfg->r_lo) || !finite(cfg->r_hi)))
        return FABRIC_E_INVAL;
    if (ctx->n_mats == 0)
        return FABRIC_E_STATE;
    return FABRIC_OK;
}

TrainArgs train_args(fabric_ctx *ctx, const fabric_gbuffer *batch, const float *targets,
                     const fabric_train_cfg *cfg)
{
    TrainArgs a;
    a.params = ctx->params;
    a.adam_m = ctx->adam_m;
    a.adam_v = ctx->adam_v;
    a.clock = AdamClock{ctx->adam_t, ctx->adam_corr};
    a.fabrics = ctx->fabrics;
    a.enc_inputs = ctx->enc_inputs;
    a.n_fabrics = ctx->n_mats;
    a.batch = batch;
    a.targets = targets;
    a.cfg = *cfg;
    a.err = ctx->err;
    a.vis = VisArgs{nullptr, nullptr};
    return a;
}
}  // namespace

fabric_status fabric_loss_grad(fabric_ctx *ctx, const fabric_gbuffer *batch, const float *targets,
                               const fabric_train_cfg *cfg, float *grad, float *out_loss,
                               void *stream)
{
    fabric_status st = check_train_args(ctx, batch, targets, cfg);
    if (st != FABRIC_OK)
        return st;
    if (!grad)
        return FABRIC_E_INVAL;
    DeviceGuard guard(ctx->device);
    TrainArgs a = train_args(ctx, batch, targets, cfg);
    if (!targets && (st = ensure_vis(ctx, as_stream(stream), &a.vis)) != FABRIC_OK)
        return st;
    return from_hip(loss_grad(ctx->train, a, grad, out_loss, as_stream(stream)));
}

fabric_status fabric_train_step(fabric_ctx *ctx, const fabric_gbuffer *batch, const float *targets,
                                const fabric_train_cfg *cfg, float *out_loss, void *stream)
{
    fabric_status st = check_train_args(ctx, batch, targets, cfg);
    if (st != FABRIC_OK)
        return st;
    DeviceGuard guard(ctx->device);
    TrainArgs a = train_args(ctx, batch, targets, cfg);
    if (!targets && (st = ensure_vis(ctx, as_stream(stream), &a.vis)) != FABRIC_OK)
        return st;
    int updated = 0;
    hipError_t e = train_step(ctx->train, a, out_loss, &updated, as_stream(stream));
    if (e != hipSuccess)
        return from_hip(e);
    ctx->weights_version += 1;
    if (!updated)
        return FABRIC_E_NONFINITE;
    return FABRIC_OK;
}

namespace {
fabric_status check_paper_train_args(fabric_ctx *ctx, const fabric_gbuffer *batch,
                                     const float *targets, const fabric_train_cfg *cfg)
{
    fabric_status st = check_train_args(ctx, batch, targets, cfg);
    if (st != FABRIC_OK)
        return st;
    if (cfg->prec != FABRIC_FP32 && cfg->prec != FABRIC_BF16)
        return FABRIC_E_INVAL;
    if (ctx->paper_n_mats == 0 || ctx->paper_serial != ctx->table_serial ||
        ctx->paper_n_mats != ctx->n_mats)
        return FABRIC_E_STATE;
    if (ctx->n_mats > kPaperTrainMaxFabrics)
        return FABRIC_E_RANGE;
    return FABRIC_OK;
}

PaperTrainArgs paper_train_args(fabric_ctx *ctx, const fabric_gbuffer *batch, const float *targets,
                                const fabric_train_cfg *cfg)
{
    PaperTrainArgs a;
    a.master = ctx->paper_master;
    a.adam_m = ctx->paper_m;
    a.adam_v = ctx->paper_v;
    a.clock = AdamClock{ctx->adam_t + 1, ctx->adam_corr + 2};
    a.fabrics = ctx->fabrics;
    a.n_fabrics = ctx->n_mats;
    a.batch = batch;
    a.targets = targets;
    a.cfg = *cfg;
    a.err = ctx->err;
    a.vis = VisArgs{nullptr, nullptr};
    a.raw = ctx->paper_raw;
    a.fused = ctx->paper_fused;
    a.enc_inputs = ctx->paper_encoder ? ctx->enc_inputs : nullptr;
    // The BF16 shading image (first in the paper image) and c_f were packed
    // from the current masters and latents by the last prepare or step.
    a.bf16_image = ctx->paper_image;
    a.cfold = ctx->paper_cfold;
    return a;
}
}  // namespace

fabric_status fabric_paper_set_footprint_encoding(fabric_ctx *ctx, int32_t one_blob)
{
    if (!ctx || (one_blob != 0 && one_blob != 1))
        return FABRIC_E_INVAL;
    ctx->paper_raw = one_blob == 0;
    return FABRIC_OK;
}

fabric_status fabric_paper_set_spatial_fusion(fabric_ctx *ctx, int32_t fused, void *stream)
{
    if (!ctx || (fused != 0 && fused != 1))
        return FABRIC_E_INVAL;
    ctx->paper_fused = fused != 0;
    if (ctx->paper_n_mats == 0 || !ctx->paper_master)
        return FABRIC_OK;
    // The shading image of the prepared masters follows the wiring.
    DeviceGuard guard(ctx->device);
    return from_hip(launch_paper_prepare(ctx->paper_master, paper_latents_of(ctx),
                                         ctx->paper_n_mats, ctx->paper_fused, ctx->paper_image,
                                         ctx->paper_cfold, as_stream(stream)));
}

fabric_status fabric_paper_loss_grad(fabric_ctx *ctx, const fabric_gbuffer *batch,
                                     const float *targets, const fabric_train_cfg *cfg, float *grad,
                                     float *out_loss, void *stream)
{
    fabric_status st = check_paper_train_args(ctx, batch, targets, cfg);
    if (st != FABRIC_OK)
        return st;
    if (!grad)
        return FABRIC_E_INVAL;
    DeviceGuard guard(ctx->device);
    PaperTrainArgs a = paper_train_args(ctx, batch, targets, cfg);
    if (!targets && (st = ensure_vis(ctx, as_stream(stream), &a.vis)) != FABRIC_OK)
        return st;
    return from_hip(paper_loss_grad(ctx->paper_train, a, grad, out_loss, as_stream(stream)));
}

fabric_status fabric_paper_train_step(fabric_ctx *ctx, const fabric_gbuffer *batch,
                                      const float *targets, const fabric_train_cfg *cfg,
                                      float *out_loss, void *stream)
{
    fabric_status st = check_paper_train_args(ctx, batch, targets, cfg);
    if (st != FABRIC_OK)
        return st;
    DeviceGuard guard(ctx->device);
    hipStream_t s = as_stream(stream);
    PaperTrainArgs a = paper_train_args(ctx, batch, targets, cfg);
    if (!targets && (st = ensure_vis(ctx, s, &a.vis)) != FABRIC_OK)
        return st;
    int updated = 0;
    hipError_t e = paper_train_step(ctx->paper_train, a, out_loss, &updated, s);
    // The shading image follows the masters (unchanged when the step was skipped).
    // With the encoder, its latents after the step (left in the training
    // scratch) become the context's.
    if (e == hipSuccess && ctx->paper_encoder)
        e = hipMemcpyAsync(ctx->paper_latents, ctx->paper_train.lat,
                           (size_t)ctx->n_mats * FABRIC_PAPER_LATENT * sizeof(float),
                           hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
        e = launch_paper_prepare(ctx->paper_master, paper_latents_of(ctx), ctx->n_mats,
                                 ctx->paper_fused, ctx->paper_image, ctx->paper_cfold, s);
    if (e != hipSuccess)
        return from_hip(e);
    if (!updated)
        return FABRIC_E_NONFINITE;
    return FABRIC_OK;
}

fabric_status fabric_paper_get_params(fabric_ctx *ctx, float *params_host, float *latents_host)
{
    if (!ctx || !params_host || !latents_host)
        return FABRIC_E_INVAL;
    if (ctx->paper_n_mats == 0 || !ctx->paper_master)
        return FABRIC_E_STATE;
    DeviceGuard guard(ctx->device);
    fabric_status st = from_hip(hipDeviceSynchronize());
    if (st == FABRIC_OK)
        st = from_hip(hipMemcpy(params_host, ctx->paper_master,
                                FABRIC_N_PAPER_DECODER_PARAMS * sizeof(float), hipMemcpyDeviceToHost));
    if (st == FABRIC_OK)
        st = from_hip(hipMemcpy(latents_host, paper_latents_of(ctx),
                                (size_t)ctx->paper_n_mats * FABRIC_PAPER_LATENT * sizeof(float),
                                hipMemcpyDeviceToHost));
    return st;
}

fabric_status fabric_get_params(fabric_ctx *ctx, float *host, size_t count)
{
    if (!ctx || !host || count != (size_t)FABRIC_N_PARAMS)
        return FABRIC_E_INVAL;
    DeviceGuard guard(ctx->device);
    fabric_status st = from_hip(hipDeviceSynchronize());
    if (st == FABRIC_OK)
        st = from_hip(hipMemcpy(host, ctx->params, count * sizeof(float), hipMemcpyDeviceToHost));
    return st;
}

fabric_status fabric_set_params(fabric_ctx *ctx, const float *host, size_t count)
{
    if (!ctx || !host || count != (size_t)FABRIC_N_PARAMS)
        return FABRIC_E_INVAL;
    for (size_t k = 0; k < count; k++)
        if (!std::isfinite(host[k]))
            return FABRIC_E_INVAL;
    DeviceGuard guard(ctx->device);
    fabric_status st = from_hip(hipDeviceSynchronize());
    if (st == FABRIC_OK)
        st = from_hip(hipMemcpy(ctx->params, host, count * sizeof(float), hipMemcpyHostToDevice));
    if (st == FABRIC_OK)
        ctx->weights_version += 1;
    return st;
}

fabric_status fabric_get_latents(fabric_ctx *ctx, float *host, int32_t n_mats)
{
    if (!ctx || !host)
        return FABRIC_E_INVAL;
    if (ctx->n_mats == 0)
        return FABRIC_E_STATE;
    if (n_mats != ctx->n_mats)
        return FABRIC_E_INVAL;
    DeviceGuard guard(ctx->device);
    fabric_status st = from_hip(hipDeviceSynchronize());
    if (st == FABRIC_OK)
        st = from_hip(hipMemcpy(host, ctx->latents, (size_t)n_mats * kLatent * sizeof(float),
                                hipMemcpyDeviceToHost));
    return st;
}

namespace {
const char kMagic[8] = {'F', 'A', 'B', 'R', 'I', 'C', 'K', '1'};
struct CkptHeader {
    char magic[8];
    uint32_t version;
    uint32_t n_params;
    int64_t step;
};
size_t ckpt_bytes()
{
    return sizeof(CkptHeader) + (size_t)FABRIC_N_PARAMS * (sizeof(float) + 2 * sizeof(double));
}
}  // namespace

fabric_status fabric_save(fabric_ctx *ctx, void *host, size_t *bytes)
{
    if (!ctx || !bytes)
        return FABRIC_E_INVAL;
    const size_t need = ckpt_bytes();
    if (!host) {
        *bytes = need;
        return FABRIC_OK;
    }
    if (*bytes < need)
        return FABRIC_E_RANGE;
    DeviceGuard guard(ctx->device);
    CkptHeader h;
    std::memcpy(h.magic, kMagic, 8);
    h.version = 1;
    h.n_params = FABRIC_N_PARAMS;
    fabric_status st = from_hip(hipDeviceSynchronize());
    if (st == FABRIC_OK)
        st = from_hip(hipMemcpy(&h.step, ctx->adam_t, sizeof(int64_t), hipMemcpyDeviceToHost));
    char *p = (char *)host;
    std::memcpy(p, &h, sizeof(h));
    p += sizeof(h);
    if (st == FABRIC_OK)
        st = from_hip(hipMemcpy(p, ctx->params, FABRIC_N_PARAMS * sizeof(float), hipMemcpyDeviceToHost));
    p += FABRIC_N_PARAMS * sizeof(float);
    if (st == FABRIC_OK)
        st = from_hip(hipMemcpy(p, ctx->adam_m, FABRIC_N_PARAMS * sizeof(double), hipMemcpyDeviceToHost));
    p += FABRIC_N_PARAMS * sizeof(double);
    if (st == FABRIC_OK)
        st = from_hip(hipMemcpy(p, ctx->adam_v, FABRIC_N_PARAMS * sizeof(double), hipMemcpyDeviceToHost));
    *bytes = need;
    return st;
}

fabric_status fabric_load(fabric_ctx *ctx, const void *host, size_t bytes)
{
    if (!ctx || !host || bytes < ckpt_bytes())
        return FABRIC_E_INVAL;
    CkptHeader h;
    std::memcpy(&h, host, sizeof(h));
    if (std::memcmp(h.magic, kMagic, 8) != 0 || h.version != 1 || h.n_params != FABRIC_N_PARAMS ||
        h.step < 0)
        return FABRIC_E_INVAL;
    DeviceGuard guard(ctx->device);
    const char *p = (const char *)host + sizeof(h);
    fabric_status st = from_hip(hipDeviceSynchronize());
    if (st == FABRIC_OK)
        st = from_hip(hipMemcpy(ctx->params, p, FABRIC_N_PARAMS * sizeof(float), hipMemcpyHostToDevice));
    p += FABRIC_N_PARAMS * sizeof(float);
    if (st == FABRIC_OK)
        st = from_hip(hipMemcpy(ctx->adam_m, p, FABRIC_N_PARAMS * sizeof(double), hipMemcpyHostToDevice));
    p += FABRIC_N_PARAMS * sizeof(double);
    if (st == FABRIC_OK)
        st = from_hip(hipMemcpy(ctx->adam_v, p, FABRIC_N_PARAMS * sizeof(double), hipMemcpyHostToDevice));
    if (st == FABRIC_OK)
        st = from_hip(hipMemcpy(ctx->adam_t, &h.step, sizeof(int64_t), hipMemcpyHostToDevice));
    if (st == FABRIC_OK)
        ctx->weights_version += 1;
    return st;
}

int64_t fabric_error_count(fabric_ctx *ctx, int reset)
{
    if (!ctx)
        return -1;
    DeviceGuard guard(ctx->device);
    unsigned long long v = 0;
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(&v, ctx->err, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess)
        return -1;
    if (reset && hipMemset(ctx->err, 0, sizeof(v)) != hipSuccess)
        return -1;
    return (int64_t)v;
}

}  // extern "C"
