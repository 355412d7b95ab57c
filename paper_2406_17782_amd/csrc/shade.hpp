// Pieces shared by the neural shading kernels (Sec. 4.3): G-buffer loads,
// per-fabric constants in LDS, and the routing of out-of-range pixels to the
// footprint filter.
#pragma once

#include "kernels.hpp"
#include "model.hpp"

namespace fab {

constexpr int kFabConsts = 16;   // per fabric in LDS: fwx fwy 1/wx 1/wy kd[2][3] ks[2][3]

// Out-of-range rule of the hybrid frame: footprint above one cell or a
// grazing view.
__device__ inline bool out_of_range(float r, float wo_z) { return r > 1.0f || wo_z < 0.05f; }

// One pixel's G-buffer fields.
struct Pix {
    int fid;
    float u, v, r;
    float3 wi, wo;
};

__device__ inline Pix load_pix(const fabric_gbuffer &g, int p)
{
    Pix x;
    x.fid = g.fabric_id[p];
    x.u = g.u[p];
    x.v = g.v[p];
    x.r = g.radius[p];
    x.wi = make_float3(g.wi_x[p], g.wi_y[p], g.wi_z[p]);
    x.wo = make_float3(g.wo_x[p], g.wo_y[p], g.wo_z[p]);
    return x;
}

// Block-cooperative fill of the per-fabric constants s_fc[n_fabrics][16].
__device__ inline void stage_fabric_consts(const DevFabric *__restrict__ fabrics, int n_fabrics,
                                           float *s_fc)
{
    for (int k = threadIdx.x; k < n_fabrics * kFabConsts; k += blockDim.x) {
        const DevFabric &f = fabrics[k / kFabConsts];
        const int c = k % kFabConsts;
        float val;
        if (c == 0) val = f.fwx;
        else if (c == 1) val = f.fwy;
        else if (c == 2) val = f.inv_wx;
        else if (c == 3) val = f.inv_wy;
        else if (c < 10) val = f.kd[(c - 4) / 3][(c - 4) % 3];
        else val = f.ks[(c - 10) / 3][(c - 10) % 3];
        s_fc[k] = val;
    }
}

// Decoded components (Eq. (8)): C = max(y, 0), S = max((e^y - 1) / 100, 0),
// composed with the fabric's albedos fc[4..15] into rgb.
template <typename FM>
__device__ inline void compose_rgb(float y0, float y1, float y2, float y3, const float *fc,
                                   float (&rgb)[3])
{
    const float cw = fmaxf(y0, 0.0f), cwf = fmaxf(y1, 0.0f);
    const float sw = fmaxf(FM::expm1(y2) * (1.0f / kSpec), 0.0f);
    const float sf = fmaxf(FM::expm1(y3) * (1.0f / kSpec), 0.0f);
#pragma unroll
    for (int c = 0; c < 3; c++)
        rgb[c] = fc[4 + c] * cw + fc[7 + c] * cwf + fc[10 + c] * sw + fc[13 + c] * sf;
}

// The analytic footprint filter for the pixels of one tile whose bits are set
// in `todo` (bit c: pixel base + c, fields held by lane c), all 64 lanes per
// pixel.  Writes rgb[3][n].
__device__ inline void shade_fallback(unsigned long long todo, int base, int n,
                                      const DevFabric *__restrict__ fabrics, int fid, float u,
                                      float v, float r, float3 wi, float3 wo, int fb_samples,
                                      int fb_side, float fb_inv_side, uint64_t seed, int lane,
                                      float *__restrict__ out)
{
    while (todo) {
        const int c = __builtin_ctzll(todo);
        todo &= todo - 1;
        const int pp = base + c;
        const int ff = __shfl(fid, c, 64);
        const float uu = __shfl(u, c, 64), vv = __shfl(v, c, 64), rr = __shfl(r, c, 64);
        const float3 wwi = make_float3(__shfl(wi.x, c, 64), __shfl(wi.y, c, 64),
                                       __shfl(wi.z, c, 64));
        const float3 wwo = make_float3(__shfl(wo.x, c, 64), __shfl(wo.y, c, 64),
                                       __shfl(wo.z, c, 64));
        double comp[4];
        filter_pixel_wave(fabrics[ff], seed, (uint64_t)pp, fb_samples, fb_side, fb_inv_side, uu,
                          vv, rr, wwi, wwo, lane, comp);
        if (lane == 0) {
            const DevFabric &f = fabrics[ff];
            for (int ch = 0; ch < 3; ch++) {
                const double rgb = (double)f.kd[0][ch] * comp[0] + (double)f.kd[1][ch] * comp[1] +
                                   (double)f.ks[0][ch] * comp[2] + (double)f.ks[1][ch] * comp[3];
                out[ch * n + pp] = (float)rgb;
            }
        }
    }
}

// Compute units of the current device (cached).
int device_cus();

// Side of the square sample grid for n footprint samples.
inline int sample_side(int n_samples)
{
    int side = 1;
    while (side * side < n_samples)
        side++;
    return side;
}

}  // namespace fab
