// Pieces shared by the neural shading kernels (Sec. 4.3): G-buffer loads,
// per-fabric constants in LDS, and the marking of out-of-range pixels for
// the footprint filter.
#pragma once

#include "kernels.hpp"
#include "model.hpp"

namespace fab {

constexpr int kFabConsts = 16;   // per fabric in LDS: fwx fwy 1/wx 1/wy kd[2][3] ks[2][3]
// The staged constants hold two copies of the fabric table: entries
// 0 .. n-1 with the specular albedos divided by k = 100 (reflection), entries
// n .. 2n-1 divided by k = 1000 (transmission, wi.z < 0).
constexpr int kFabCopies = 2;

// Staged-constant entry of fabric fid for a pixel lit from below or above.
__device__ inline int fab_entry(int fid, int n_fabrics, float wi_z)
{
    return wi_z < 0.0f ? fid + n_fabrics : fid;
}

// Out-of-range rule of the hybrid frame: footprint above one cell or a
// grazing view.
__device__ inline bool out_of_range(float r, float wo_z) { return r > 1.0f || wo_z < 0.05f; }

// One pixel's G-buffer fields.
struct Pix {
    int fid;
    float u, v, r;
    float3 wi, wo;
};

// Element i of a G-buffer plane through a 32-bit byte offset from the
// plane's base, which lets the load use the scalar-base + vector-offset
// address form (no 64-bit address arithmetic per lane).  Valid because the
// boundary limits n to INT32_MAX / 16, so 12 n bytes stay below 2^32.
template <typename T> __device__ inline T plane_at(const T *base, int i)
{
    return *(const T *)((const char *)base + (uint32_t)i * (uint32_t)sizeof(T));
}
__device__ inline void plane_store(float *base, int i, float v)
{
    *(float *)((char *)base + (uint32_t)i * 4u) = v;
}

__device__ inline Pix load_pix(const fabric_gbuffer &g, int p)
{
    Pix x;
    x.fid = plane_at(g.fabric_id, p);
    x.u = plane_at(g.u, p);
    x.v = plane_at(g.v, p);
    x.r = plane_at(g.radius, p);
    x.wi = make_float3(plane_at(g.wi_x, p), plane_at(g.wi_y, p), plane_at(g.wi_z, p));
    x.wo = make_float3(plane_at(g.wo_x, p), plane_at(g.wo_y, p), plane_at(g.wo_z, p));
    return x;
}

// The half of a pixel's fields one lane group of a 32-pixel tile needs:
// group 0 the u coordinate and wi, group 1 v and wo; both the radius and the
// fabric id.  Six loads per lane instead of ten.
struct HalfPix {
    int fid;
    float uv, r;
    float x0, x1, xz;   // (wi or wo).x, .y, .z
};
struct HalfPlanes {
    const float *uv, *x0, *x1, *xz;
};
__device__ inline HalfPlanes half_planes(const fabric_gbuffer &g, int grp)
{
    HalfPlanes h;
    h.uv = grp ? g.v : g.u;
    h.x0 = grp ? g.wo_x : g.wi_x;
    h.x1 = grp ? g.wo_y : g.wi_y;
    h.xz = grp ? g.wo_z : g.wi_z;
    return h;
}
__device__ inline HalfPix load_half(const fabric_gbuffer &g, const HalfPlanes &h, int p)
{
    HalfPix x;
    x.fid = plane_at(g.fabric_id, p);
    x.r = plane_at(g.radius, p);
    x.uv = h.uv[p];
    x.x0 = h.x0[p];
    x.x1 = h.x1[p];
    x.xz = h.xz[p];
    return x;
}
// This lane group's share of the fault rule of pixel_fault (group 0 holds
// wi, which may point below the fabric, group 1 wo), as a lane mask: one
// comparison per condition, combined on the scalar unit.  The direction rule
// is !(z' > 0) with z' = wo.z in group 1 and |wi.z| in group 0 (dir_mask of
// half_dir_mask clears the sign there).
__device__ inline uint32_t half_dir_mask(int grp) { return grp ? 0xffffffffu : 0x7fffffffu; }
__device__ inline unsigned long long half_fault(const HalfPix &x, int n_fabrics, uint32_t dir_mask)
{
    const float zsel = __uint_as_float(__float_as_uint(x.xz) & dir_mask);
    return __ballot(!isfinite(x.uv)) | __ballot(!isfinite(x.r)) | __ballot(!isfinite(x.x0)) |
           __ballot(!isfinite(x.x1)) | __ballot(!isfinite(x.xz)) | __ballot(x.fid >= n_fabrics) |
           __ballot(!(x.r > 0.0f)) | __ballot(!(zsel > 0.0f));
}
// Lane mask with both lanes of a pixel (lanes l and l ^ 32) set when either
// lane's bit of m is set.
__device__ inline unsigned long long pair_mask(unsigned long long m)
{
    return m | (m >> 32) | (m << 32);
}
// This lane's bit of pair_mask(m).
__device__ inline bool pair_any(unsigned long long m)
{
    return __builtin_amdgcn_inverse_ballot_w64(pair_mask(m));
}
__device__ inline bool pair_any(bool flag) { return pair_any(__ballot(flag)); }

// Block-cooperative fill of the per-fabric constants s_fc[2 n_fabrics][16]:
// fwx, fwy, 1/wx, 1/wy, kd (warp, weft RGB), ks / k (warp, weft RGB).  The
// specular albedos carry the 1/k of the decoding S = (e^y - 1) / k: k = 100
// in the first copy, 1000 in the second (transmission, Sec. 4.2).
__device__ inline void stage_fabric_consts(const DevFabric *__restrict__ fabrics, int n_fabrics,
                                           float *s_fc)
{
    for (int k = threadIdx.x; k < kFabCopies * n_fabrics * kFabConsts; k += blockDim.x) {
        const int entry = k / kFabConsts;
        const bool transmit = entry >= n_fabrics;
        const DevFabric &f = fabrics[transmit ? entry - n_fabrics : entry];
        const int c = k % kFabConsts;
        float val;
        if (c == 0) val = f.fwx;
        else if (c == 1) val = f.fwy;
        else if (c == 2) val = f.inv_wx;
        else if (c == 3) val = f.inv_wy;
        else if (c < 10) val = f.kd[(c - 4) / 3][(c - 4) % 3];
        else val = f.ks[(c - 10) / 3][(c - 10) % 3] * (transmit ? 0.1f / kSpec : 1.0f / kSpec);
        s_fc[k] = val;
    }
}

// max(x, 0) as one signed-integer max of the bits (a negative float is a
// negative int32; -0 gives +0).
__device__ inline float relu_bits(float x)
{
    return __int_as_float(max(__float_as_int(x), 0));
}

// Decoded components (Eq. (8)): C = max(y, 0), S = max((e^y - 1) / k, 0)
// with k = 100 for reflection and 1000 for transmission (Sec. 4.2), composed
// with the albedos fc[4..15] of the pixel's staged entry into rgb (the 1/k
// of S is folded into the entry's specular albedos).
template <typename FM>
__device__ inline void compose_rgb(float y0, float y1, float y2, float y3, const float *fc,
                                   float (&rgb)[3])
{
    const float cw = relu_bits(y0), cwf = relu_bits(y1);
    const float sw = relu_bits(FM::expm1(y2));
    const float sf = relu_bits(FM::expm1(y3));
#pragma unroll
    for (int c = 0; c < 3; c++)
        rgb[c] = fc[4 + c] * cw + fc[7 + c] * cwf + fc[10 + c] * sw + fc[13 + c] * sf;
}

// Record the out-of-range pixels of one tile (bit c of `bits`: pixel
// 16 * group + c) in the fallback queue's mask: 16 pixels per entry, written
// by lane 0.
__device__ inline void queue_mark16(uint32_t bits, int group, FallbackQueue q, int lane)
{
    if (lane == 0)
        q.mask[group] = (uint16_t)bits;
}
// The same for a 32-pixel tile (two mask entries in one 32-bit store).
__device__ inline void queue_mark32(uint32_t bits, int tile, FallbackQueue q, int lane)
{
    if (lane == 0)
        ((uint32_t *)q.mask)[tile] = bits;
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
