// Training of the paper-size decoder (Sec. 4.2 "Decoder"; loss of Eq. (9)-(11))
// with one latent of 64 per fabric trained as a parameter.
//
//   paper_fwd_bwd_kernel   one thread per sample: one-blob features, the
//                          seven layers forward in FP32 (inputs in registers,
//                          each layer's outputs stored to the sample's
//                          planes), the loss terms and dL/dy, then the
//                          layers backward (transposed weights), storing
//                          every layer's gradient at its pre-activation
//   paper_wgrad_kernel     split-K weight gradients: per (job, chunk of
//                          1,024 samples) block, dL/dW and dL/db of one
//                          layer as sums of outer products over the chunk,
//                          staged through LDS 32 samples at a time; one job
//                          sums F1's input gradient per fabric instead
//   paper_wgrad_reduce_kernel  fixed-order sum over the chunks
//   paper_latent_grads_kernel  F1's latent columns and the latents'
//                          gradients from the per-fabric sums
// Every reduction has a fixed order: results do not depend on scheduling.
#include <cmath>

#include "kernels.hpp"
#include "model.hpp"
#include "paper_net.hpp"
#include "paper_train.hpp"
#include "shade.hpp"
#include "train.hpp"

namespace fab {

namespace {

// Per-sample planes, each [cap] floats.
constexpr int kPlFeat = 0;              // 24 one-blob channels
constexpr int kPlAng = kPlFeat + 24;    // wi.xyz, wo.xy
constexpr int kPlT = kPlAng + 5;        // F1 activation (64)
constexpr int kPlSP = kPlT + 64;        // F2: the spatial feature
constexpr int kPlX = kPlSP + 64;        // A1: the residual block's input
constexpr int kPlH = kPlX + 64;         // A2
constexpr int kPlRR = kPlH + 64;        // A3 (skip added before its activation)
constexpr int kPlG = kPlRR + 64;        // A4
constexpr int kPlDY = kPlG + 64;        // dL/dy (4)
constexpr int kPlDT = kPlDY + 4;        // dL/d(pre-activation) of F1, F2, A1 .. A4
constexpr int kPlDSP = kPlDT + 64;
constexpr int kPlDX = kPlDSP + 64;
constexpr int kPlDH = kPlDX + 64;
constexpr int kPlDRR = kPlDH + 64;
constexpr int kPlDG = kPlDRR + 64;
constexpr int kPlanes = kPlDG + 64;
static_assert(kPlanes == 801, "plane count");

// Transposed 64 x 64 blocks: WT[l][i][o] = W_l[o][i].
enum { kTF2 = 0, kTA1, kTA2, kTA3, kTA4, kTLayers };

__global__ void transpose_kernel(const float *__restrict__ P, float *__restrict__ wt)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= kTLayers * 64 * 64)
        return;
    const int l = idx / 4096, i = (idx / 64) % 64, o = idx % 64;
    const int off = l == kTF2 ? kPOffWF2 : l == kTA1 ? kPOffWA1 : l == kTA2 ? kPOffWA2
                    : l == kTA3 ? kPOffWA3 : kPOffWA4;
    const int row = l == kTA1 ? kPXA1 : 64;
    wt[idx] = P[off + o * row + i];
}

// One-blob channels of the footprint (FP32, library functions): circular
// position bins along u and v, then size bins.  raw (the encoding's
// ablation): p_u, p_v and tau in channels 0, 8 and 16, zeros elsewhere.
__device__ inline void blob24(const DevFabric &f, float u, float v, float r, bool raw,
                              float (&x)[24])
{
    const float p[2] = {wrap_period(u, f.fwx, f.inv_wx) * f.inv_wx,
                        wrap_period(v, f.fwy, f.inv_wy) * f.inv_wy};
    if (raw) {
#pragma unroll
        for (int k = 0; k < 24; k++)
            x[k] = 0.0f;
        x[0] = p[0];
        x[8] = p[1];
        x[16] = fminf(fmaxf((log2f(r) + 14.0f) * (1.0f / 16.0f), 0.0f), 1.0f);
        return;
    }
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 8; b++) {
            float d = 8.0f * p[a] - ((float)b + 0.5f);
            d -= 8.0f * floorf((d + 4.0f) * 0.125f);
            x[8 * a + b] = expf(-0.5f * d * d);
        }
    const float tau = fminf(fmaxf((log2f(r) + 14.0f) * (1.0f / 16.0f), 0.0f), 1.0f);
#pragma unroll
    for (int b = 0; b < 8; b++) {
        const float d = 8.0f * tau - ((float)b + 0.5f);
        x[16 + b] = expf(-0.5f * d * d);
    }
}

template <int N>
__device__ inline void load_vec(const float *__restrict__ pl, int plane, int64_t cap, int64_t s,
                                float (&x)[N])
{
#pragma unroll
    for (int k = 0; k < N; k++)
        x[k] = pl[(int64_t)(plane + k) * cap + s];
}

// out = lrelu(W x + b [+ skip]) for a 64-output layer whose rows hold NIN
// inputs; outputs go to the sample's planes.
template <int NIN>
__device__ inline void layer_fwd(const float *__restrict__ W, const float *__restrict__ b,
                                 const float (&x)[NIN], float *__restrict__ pl, int skip_plane,
                                 int out_plane, int64_t cap, int64_t s)
{
#pragma unroll 2
    for (int o = 0; o < 64; o++) {
        float acc = b[o];
#pragma unroll
        for (int i = 0; i < NIN; i++)
            acc = fmaf(W[o * NIN + i], x[i], acc);
        if (skip_plane >= 0)
            acc += pl[(int64_t)(skip_plane + o) * cap + s];
        pl[(int64_t)(out_plane + o) * cap + s] = lrelu(acc);
    }
}

// d_i = slope(act_i) (sum_o W[o][i] g_o [+ extra_i]) for i < 64, with the
// weight of (o, i) at W[o * SO + i * SI]; stored to the gradient plane.
template <int NG, int SO, int SI>
__device__ inline void layer_bwd(const float *__restrict__ W, const float (&gin)[NG],
                                 float *__restrict__ pl, int act_plane, int extra_plane,
                                 int out_plane, int64_t cap, int64_t s)
{
#pragma unroll 2
    for (int i = 0; i < 64; i++) {
        float acc = 0.0f;
#pragma unroll
        for (int o = 0; o < NG; o++)
            acc = fmaf(W[o * SO + i * SI], gin[o], acc);
        if (extra_plane >= 0)
            acc += pl[(int64_t)(extra_plane + i) * cap + s];
        const float a = pl[(int64_t)(act_plane + i) * cap + s];
        pl[(int64_t)(out_plane + i) * cap + s] = a > 0.0f ? acc : kLeak * acc;
    }
}

__global__ __launch_bounds__(256) void paper_fwd_bwd_kernel(
    fabric_gbuffer g, const DevFabric *__restrict__ fabrics, int n_fabrics,
    const float *__restrict__ P, const float *__restrict__ lat, const float *__restrict__ wt,
    const float *__restrict__ targets, float *__restrict__ pl, int64_t cap, int raw,
    double *__restrict__ loss_part)
{
    __shared__ double red[256];
    const int64_t n = g.n;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double loss = 0.0;
    if (s < n) {
        const int fid = g.fabric_id[s];
        const float u = g.u[s], v = g.v[s], r = g.radius[s];
        const float3 wi = make_float3(g.wi_x[s], g.wi_y[s], g.wi_z[s]);
        const float3 wo = make_float3(g.wo_x[s], g.wo_y[s], g.wo_z[s]);
        if (pixel_fault(fid, n_fabrics, u, v, r, wi, wo)) {
            // Contributes nothing: zero activations and gradients alike.
            for (int k = 0; k < kPlanes; k++)
                pl[(int64_t)k * cap + s] = 0.0f;
        } else {
            // ---- forward ----
            {
                float x1[kPX1];
#pragma unroll
                for (int k = 0; k < kPLat; k++)
                    x1[k] = lat[fid * kPLat + k];
                float f[24];
                blob24(fabrics[fid], u, v, r, raw != 0, f);
#pragma unroll
                for (int k = 0; k < 24; k++) {
                    x1[kPLat + k] = f[k];
                    pl[(int64_t)(kPlFeat + k) * cap + s] = f[k];
                }
                layer_fwd<kPX1>(P + kPOffWF1, P + kPOffBF1, x1, pl, -1, kPlT, cap, s);
            }
            {
                float x[64];
                load_vec(pl, kPlT, cap, s, x);
                layer_fwd<64>(P + kPOffWF2, P + kPOffBF2, x, pl, -1, kPlSP, cap, s);
            }
            {
                float x[kPXA1];
                float sp[64];
                load_vec(pl, kPlSP, cap, s, sp);
#pragma unroll
                for (int k = 0; k < 64; k++)
                    x[k] = sp[k];
                const float ang[5] = {wi.x, wi.y, wi.z, wo.x, wo.y};
#pragma unroll
                for (int k = 0; k < 5; k++) {
                    x[64 + k] = ang[k];
                    pl[(int64_t)(kPlAng + k) * cap + s] = ang[k];
                }
                layer_fwd<kPXA1>(P + kPOffWA1, P + kPOffBA1, x, pl, -1, kPlX, cap, s);
            }
            {
                float x[64];
                load_vec(pl, kPlX, cap, s, x);
                layer_fwd<64>(P + kPOffWA2, P + kPOffBA2, x, pl, -1, kPlH, cap, s);
            }
            {
                float x[64];
                load_vec(pl, kPlH, cap, s, x);
                layer_fwd<64>(P + kPOffWA3, P + kPOffBA3, x, pl, kPlX, kPlRR, cap, s);
            }
            {
                float x[64];
                load_vec(pl, kPlRR, cap, s, x);
                layer_fwd<64>(P + kPOffWA4, P + kPOffBA4, x, pl, -1, kPlG, cap, s);
            }
            float y[4];
            {
                float x[64];
                load_vec(pl, kPlG, cap, s, x);
#pragma unroll
                for (int o = 0; o < 4; o++) {
                    float acc = P[kPOffBA5 + o];
#pragma unroll
                    for (int i = 0; i < 64; i++)
                        acc = fmaf(P[kPOffWA5 + o * 64 + i], x[i], acc);
                    y[o] = acc;
                }
            }
            // ---- loss terms of Eq. (9)-(11) and dL/dy ----
            float dy[4];
            {
                const float inv_n = 1.0f / (float)n;
                // g(x) = ln(k x + 1): k = 100 for reflection, 1000 for transmission.
                const float k = wi.z < 0.0f ? 10.0f * kSpec : kSpec;
#pragma unroll
                for (int c = 0; c < 4; c++) {
                    const float t = targets[c * n + s];
                    const float target = c < 2 ? t : log1pf(k * t);
                    const float lam = c < 2 ? 0.1f : 0.4f;        // lambda_C, lambda_S
                    const float d = y[c] - target;
                    loss += (double)(lam * d * d);
                    dy[c] = 2.0f * lam * d * inv_n;
                    pl[(int64_t)(kPlDY + c) * cap + s] = dy[c];
                }
            }
            // ---- backward ----
            layer_bwd<4, 64, 1>(P + kPOffWA5, dy, pl, kPlG, -1, kPlDG, cap, s);
            {
                float gv[64];
                load_vec(pl, kPlDG, cap, s, gv);
                layer_bwd<64, 1, 64>(wt + kTA4 * 4096, gv, pl, kPlRR, -1, kPlDRR, cap, s);
            }
            {
                float gv[64];
                load_vec(pl, kPlDRR, cap, s, gv);
                layer_bwd<64, 1, 64>(wt + kTA3 * 4096, gv, pl, kPlH, -1, kPlDH, cap, s);
            }
            {
                // The skip carries A3's pre-activation gradient to A1's output.
                float gv[64];
                load_vec(pl, kPlDH, cap, s, gv);
                layer_bwd<64, 1, 64>(wt + kTA2 * 4096, gv, pl, kPlX, kPlDRR, kPlDX, cap, s);
            }
            {
                float gv[64];
                load_vec(pl, kPlDX, cap, s, gv);
                layer_bwd<64, 1, 64>(wt + kTA1 * 4096, gv, pl, kPlSP, -1, kPlDSP, cap, s);
            }
            {
                float gv[64];
                load_vec(pl, kPlDSP, cap, s, gv);
                layer_bwd<64, 1, 64>(wt + kTF2 * 4096, gv, pl, kPlT, -1, kPlDT, cap, s);
            }
        }
    }
    red[threadIdx.x] = loss;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        loss_part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void paper_loss_reduce_kernel(const double *__restrict__ part,
                                                                int64_t nparts, double inv_n,
                                                                double *__restrict__ loss)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t k = threadIdx.x; k < nparts; k += blockDim.x)
        acc += part[k];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        loss[0] = red[0] * inv_n;
}

// ---- split-K weight gradients ----------------------------------------------

// One job: out[i][j] = sum_s delta_i(s) in_j(s) over i < n_out and the
// inputs [planes inA .. inA + nA, inB .. inB + nB, then 1 for the bias when
// b_off >= 0]; or, for the one-hot job, in_j(s) = [fabric id of s == j].
struct PWJob {
    int delta, n_out, inA, nA, inB, nB;
    int w_off, row, col, b_off;     // destination in the parameter gradient
    int onehot;                     // 1: per-fabric sums into dsum[j][i]
};
constexpr int kPWMaxJobs = 8;
struct PWJobs {
    PWJob j[kPWMaxJobs];
    int64_t poff[kPWMaxJobs];       // job offsets in the partial buffer
    int n_jobs;
};

constexpr int kPwSub = 32;          // samples per LDS sub-tile
constexpr int kPwChunk = 1024;      // samples per block
constexpr int kPwMaxIn = 70;        // columns (inputs + bias) of any job
constexpr int kPwMaxE = 18;         // entries per thread: 64 x 70 <= 256 x 18

__host__ __device__ inline int pw_cols(const PWJob &jb)
{
    return jb.nA + jb.nB + (jb.b_off >= 0 ? 1 : 0);
}

__global__ __launch_bounds__(256) void paper_wgrad_kernel(PWJobs jobs, const float *__restrict__ pl,
                                                          int64_t cap, const uint16_t *__restrict__ fid,
                                                          int64_t n, float *__restrict__ partial)
{
    __shared__ float dt[64][kPwSub + 1];
    __shared__ float it[kPwMaxIn][kPwSub + 1];
    const PWJob jb = jobs.j[blockIdx.y];
    const int cols = pw_cols(jb);
    const int E = jb.n_out * cols;
    float acc[kPwMaxE];
#pragma unroll
    for (int m = 0; m < kPwMaxE; m++)
        acc[m] = 0.0f;
    const int64_t s0 = (int64_t)blockIdx.x * kPwChunk;
    const int64_t s1 = s0 + kPwChunk < n ? s0 + kPwChunk : n;
    for (int64_t sb = s0; sb < s1; sb += kPwSub) {
        for (int k = threadIdx.x; k < jb.n_out * kPwSub; k += blockDim.x) {
            const int i = k / kPwSub, q = k % kPwSub;
            const int64_t s = sb + q;
            dt[i][q] = s < s1 ? pl[(int64_t)(jb.delta + i) * cap + s] : 0.0f;
        }
        for (int k = threadIdx.x; k < cols * kPwSub; k += blockDim.x) {
            const int j = k / kPwSub, q = k % kPwSub;
            const int64_t s = sb + q;
            float val = 0.0f;
            if (s < s1) {
                if (jb.onehot)
                    val = (int)fid[s] == j ? 1.0f : 0.0f;
                else if (j < jb.nA)
                    val = pl[(int64_t)(jb.inA + j) * cap + s];
                else if (j < jb.nA + jb.nB)
                    val = pl[(int64_t)(jb.inB + j - jb.nA) * cap + s];
                else
                    val = 1.0f;
            }
            it[j][q] = val;
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < kPwMaxE; m++) {
            const int e = threadIdx.x + 256 * m;
            if (e < E) {
                const int i = e / cols, j = e % cols;
                float a = acc[m];
#pragma unroll 8
                for (int q = 0; q < kPwSub; q++)
                    a = fmaf(dt[i][q], it[j][q], a);
                acc[m] = a;
            }
        }
        __syncthreads();
    }
    float *dst = partial + jobs.poff[blockIdx.y] + (int64_t)blockIdx.x * E;
#pragma unroll
    for (int m = 0; m < kPwMaxE; m++) {
        const int e = threadIdx.x + 256 * m;
        if (e < E)
            dst[e] = acc[m];
    }
}

__global__ __launch_bounds__(256) void paper_wgrad_reduce_kernel(PWJobs jobs, int n_chunks,
                                                                 const float *__restrict__ partial,
                                                                 float *__restrict__ grad,
                                                                 float *__restrict__ dsum)
{
    const PWJob jb = jobs.j[blockIdx.y];
    const int cols = pw_cols(jb);
    const int E = jb.n_out * cols;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E)
        return;
    const float *src = partial + jobs.poff[blockIdx.y] + e;
    double acc = 0.0;
    for (int c = 0; c < n_chunks; c++)
        acc += (double)src[(int64_t)c * E];
    const int i = e / cols, j = e % cols;
    if (jb.onehot)
        dsum[j * 64 + i] = (float)acc;
    else if (j < jb.nA + jb.nB)
        grad[jb.w_off + i * jb.row + jb.col + j] = (float)acc;
    else
        grad[jb.b_off + i] = (float)acc;
}

// F1's latent columns: dWF1[o][j] = sum_f D[f][o] z_f[j]; the latents:
// dz_f[j] = sum_o WF1[o][j] D[f][o] (D: per-fabric sums of F1's gradient).
__global__ void paper_latent_grads_kernel(const float *__restrict__ P, const float *__restrict__ lat,
                                          const float *__restrict__ dsum, int n_fabrics,
                                          float *__restrict__ grad, float *__restrict__ glat)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < 64 * kPLat) {
        const int o = idx / kPLat, j = idx % kPLat;
        float acc = 0.0f;
        for (int f = 0; f < n_fabrics; f++)
            acc = fmaf(dsum[f * 64 + o], lat[f * kPLat + j], acc);
        grad[kPOffWF1 + o * kPX1 + j] = acc;
    } else if (idx < 64 * kPLat + n_fabrics * kPLat) {
        const int k = idx - 64 * kPLat;
        const int f = k / kPLat, j = k % kPLat;
        float acc = 0.0f;
        for (int o = 0; o < 64; o++)
            acc = fmaf(P[kPOffWF1 + o * kPX1 + j], dsum[f * 64 + o], acc);
        glat[f * kPLat + j] = acc;
    }
}

template <typename Tp> hipError_t regrow(Tp **p, size_t count)
{
    (void)hipFree(*p);
    *p = nullptr;
    return hipMalloc((void **)p, count * sizeof(Tp));
}

PWJobs make_jobs(int n_fabrics, int n_chunks)
{
    PWJobs J;
    auto job = [](int delta, int n_out, int inA, int nA, int inB, int nB, int w_off, int row,
                  int col, int b_off) {
        return PWJob{delta, n_out, inA, nA, inB, nB, w_off, row, col, b_off, 0};
    };
    int k = 0;
    J.j[k++] = job(kPlDY, 4, kPlG, 64, 0, 0, kPOffWA5, 64, 0, kPOffBA5);
    J.j[k++] = job(kPlDG, 64, kPlRR, 64, 0, 0, kPOffWA4, 64, 0, kPOffBA4);
    J.j[k++] = job(kPlDRR, 64, kPlH, 64, 0, 0, kPOffWA3, 64, 0, kPOffBA3);
    J.j[k++] = job(kPlDH, 64, kPlX, 64, 0, 0, kPOffWA2, 64, 0, kPOffBA2);
    J.j[k++] = job(kPlDX, 64, kPlSP, 64, kPlAng, 5, kPOffWA1, kPXA1, 0, kPOffBA1);
    J.j[k++] = job(kPlDSP, 64, kPlT, 64, 0, 0, kPOffWF2, 64, 0, kPOffBF2);
    J.j[k++] = job(kPlDT, 64, kPlFeat, 24, 0, 0, kPOffWF1, kPX1, kPLat, kPOffBF1);
    J.j[k++] = PWJob{kPlDT, 64, 0, n_fabrics, 0, 0, 0, 0, 0, -1, 1};
    J.n_jobs = k;
    int64_t off = 0;
    for (int q = 0; q < k; q++) {
        J.poff[q] = off;
        off += (int64_t)n_chunks * J.j[q].n_out * pw_cols(J.j[q]);
    }
    return J;
}

// Loss and gradient ([params | latents], into s.grad) of one batch.
hipError_t run_paper_loss_grad(PaperTrainScratch &s, const PaperTrainArgs &a, hipStream_t stream)
{
    const fabric_train_cfg &cfg = a.cfg;
    hipError_t e;
    if (!s.grad) {
        if ((e = hipMalloc((void **)&s.grad, (size_t)(kPNDec + kPaperTrainMaxFabrics * kPLat) * sizeof(float))) != hipSuccess) return e;
        if ((e = hipMalloc((void **)&s.dsum, (size_t)kPaperTrainMaxFabrics * 64 * sizeof(float))) != hipSuccess) return e;
        if ((e = hipMalloc((void **)&s.wt, (size_t)kTLayers * 4096 * sizeof(float))) != hipSuccess) return e;
        if ((e = hipMalloc((void **)&s.loss, sizeof(double))) != hipSuccess) return e;
    }
    fabric_gbuffer g;
    if (a.batch) {
        g = *a.batch;
    } else {
        const int64_t n = cfg.batch;
        if (s.batch_cap < n) {
            if ((e = regrow(&s.b_fid, (size_t)n)) != hipSuccess) return e;
            if ((e = regrow(&s.b_fields, (size_t)n * 9)) != hipSuccess) return e;
            if ((e = regrow(&s.targets, (size_t)n * 4)) != hipSuccess) return e;
            s.batch_cap = n;
        }
        fabric_gbuffer_out o;
        o.n = n;
        o.fabric_id = s.b_fid;
        float *f = s.b_fields;
        const int64_t c = s.batch_cap;
        o.u = f; o.v = f + c; o.radius = f + 2 * c; o.wi_x = f + 3 * c; o.wi_y = f + 4 * c;
        o.wi_z = f + 5 * c; o.wo_x = f + 6 * c; o.wo_y = f + 7 * c; o.wo_z = f + 8 * c;
        if ((e = launch_make_batch(cfg.seed, n, a.n_fabrics, cfg.r_lo, cfg.r_hi, cfg.btdf_frac, o,
                                   stream)) != hipSuccess)
            return e;
        g.n = n; g.fabric_id = o.fabric_id; g.u = o.u; g.v = o.v; g.radius = o.radius;
        g.wi_x = o.wi_x; g.wi_y = o.wi_y; g.wi_z = o.wi_z; g.wo_x = o.wo_x; g.wo_y = o.wo_y; g.wo_z = o.wo_z;
    }
    const int64_t n = g.n;
    const float *P = a.master, *lat = a.master + kPNDec;
    float *grad = s.grad, *glat = s.grad + kPNDec;
    if (n == 0) {
        if ((e = hipMemsetAsync(s.loss, 0, sizeof(double), stream)) != hipSuccess) return e;
        return hipMemsetAsync(s.grad, 0, (size_t)(kPNDec + a.n_fabrics * kPLat) * sizeof(float), stream);
    }
    const float *targets = a.targets;
    if (!targets) {
        if (s.batch_cap < n) {
            // A caller-supplied batch larger than any generated one: the
            // batch planes are not in use, so all three buffers may grow.
            if ((e = regrow(&s.targets, (size_t)n * 4)) != hipSuccess) return e;
            if ((e = regrow(&s.b_fid, (size_t)n)) != hipSuccess) return e;
            if ((e = regrow(&s.b_fields, (size_t)n * 9)) != hipSuccess) return e;
            s.batch_cap = n;
        }
        if ((e = launch_gt_filter(g, a.fabrics, a.n_fabrics, cfg.gt_samples, cfg.seed ^ 1ull, a.vis,
                                  nullptr, s.targets, a.err, stream)) != hipSuccess)
            return e;
        targets = s.targets;
    }
    const int64_t blocks = (n + 255) / 256;
    if (s.cap < n) {
        if ((e = regrow(&s.planes, (size_t)n * kPlanes)) != hipSuccess) return e;
        if ((e = regrow(&s.loss_part, (size_t)blocks)) != hipSuccess) return e;
        s.cap = n;
    }
    const int n_chunks = (int)((n + kPwChunk - 1) / kPwChunk);
    const PWJobs jobs = make_jobs(a.n_fabrics, n_chunks);
    const size_t need = (size_t)(jobs.poff[jobs.n_jobs - 1] +
                                 (int64_t)n_chunks * jobs.j[jobs.n_jobs - 1].n_out *
                                     pw_cols(jobs.j[jobs.n_jobs - 1]));
    if (s.partial_floats < need) {
        if ((e = regrow(&s.partial, need)) != hipSuccess) return e;
        s.partial_floats = need;
    }
    hipLaunchKernelGGL(transpose_kernel, dim3((kTLayers * 4096 + 255) / 256), dim3(256), 0, stream,
                       P, s.wt);
    // Faults of a generated-target batch were counted by the filter.
    (void)a.err;
    hipLaunchKernelGGL(paper_fwd_bwd_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, g,
                       a.fabrics, a.n_fabrics, P, lat, (const float *)s.wt, targets, s.planes,
                       s.cap, a.raw ? 1 : 0, s.loss_part);
    hipLaunchKernelGGL(paper_loss_reduce_kernel, dim3(1), dim3(256), 0, stream,
                       (const double *)s.loss_part, blocks, 1.0 / (double)n, s.loss);
    hipLaunchKernelGGL(paper_wgrad_kernel, dim3(n_chunks, jobs.n_jobs), dim3(256), 0, stream, jobs,
                       (const float *)s.planes, s.cap, g.fabric_id, n, s.partial);
    hipLaunchKernelGGL(paper_wgrad_reduce_kernel, dim3((64 * kPwMaxIn + 255) / 256, jobs.n_jobs),
                       dim3(256), 0, stream, jobs, n_chunks, (const float *)s.partial, grad, s.dsum);
    const int tot = 64 * kPLat + a.n_fabrics * kPLat;
    hipLaunchKernelGGL(paper_latent_grads_kernel, dim3((tot + 255) / 256), dim3(256), 0, stream, P,
                       lat, (const float *)s.dsum, a.n_fabrics, grad, glat);
    return hipGetLastError();
}

hipError_t read_paper_loss(PaperTrainScratch &s, float *out_loss, int *finite_loss,
                           hipStream_t stream)
{
    double l = 0.0;
    hipError_t e;
    if ((e = hipMemcpyAsync(&l, s.loss, sizeof(double), hipMemcpyDeviceToHost, stream)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(stream)) != hipSuccess) return e;
    *out_loss = (float)l;
    *finite_loss = std::isfinite(l) ? 1 : 0;
    return hipSuccess;
}

}  // namespace

void paper_train_scratch_free(PaperTrainScratch &s)
{
    (void)hipFree(s.planes);
    (void)hipFree(s.loss_part);
    (void)hipFree(s.loss);
    (void)hipFree(s.wt);
    (void)hipFree(s.partial);
    (void)hipFree(s.grad);
    (void)hipFree(s.dsum);
    (void)hipFree(s.b_fid);
    (void)hipFree(s.b_fields);
    (void)hipFree(s.targets);
    s = PaperTrainScratch();
}

hipError_t paper_loss_grad(PaperTrainScratch &s, const PaperTrainArgs &a, float *grad_out,
                           float *out_loss, hipStream_t stream)
{
    hipError_t e = run_paper_loss_grad(s, a, stream);
    if (e != hipSuccess)
        return e;
    if ((e = hipMemcpyAsync(grad_out, s.grad, (size_t)(kPNDec + a.n_fabrics * kPLat) * sizeof(float),
                            hipMemcpyDeviceToDevice, stream)) != hipSuccess)
        return e;
    if (out_loss) {
        int fin = 0;
        return read_paper_loss(s, out_loss, &fin, stream);
    }
    return hipSuccess;
}

hipError_t paper_train_step(PaperTrainScratch &s, const PaperTrainArgs &a, float *out_loss,
                            int *updated, hipStream_t stream)
{
    *updated = 1;
    hipError_t e = run_paper_loss_grad(s, a, stream);
    if (e != hipSuccess)
        return e;
    if ((e = launch_adam(a.master, s.grad, a.adam_m, a.adam_v, kPNDec + a.n_fabrics * kPLat, a.cfg,
                         a.step, s.loss, stream)) != hipSuccess)
        return e;
    if (out_loss)
        return read_paper_loss(s, out_loss, updated, stream);
    return hipSuccess;
}

}  // namespace fab
