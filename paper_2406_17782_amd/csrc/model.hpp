// Device-side analytic fabric model in FP32: sample generation over a pixel
// footprint, the procedural yarn geometry, the point shading model of
// Eq. (1)-(2) and the per-sample integrand of the footprint aggregation
// Eq. (3)-(4) with visibility V = 1.
#pragma once

#include "common.hpp"

namespace fab {

// The index-th output of the SplitMix64 generator started at `seed`
// (Steele, Lea and Flood 2014): the state advances by the golden gamma and
// the output is the variant-13 finaliser of the new state.
constexpr uint64_t kGoldenGamma = 0x9E3779B97F4A7C15ull;

__device__ inline uint64_t splitmix64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t index)
{
    return splitmix64_mix(seed + (index + 1ull) * kGoldenGamma);
}

// Upper and middle 24-bit fields of a 64-bit draw as uniforms in [0, 1).
__device__ inline float u24_hi(uint64_t z) { return (float)(uint32_t)(z >> 40) * 0x1p-24f; }
__device__ inline float u24_mid(uint64_t z)
{
    return (float)(uint32_t)((z >> 16) & 0xFFFFFFull) * 0x1p-24f;
}

// Accurate float32 transcendentals (a few ulp) for everything that sets a
// sample's position or its ply frame: an error there moves the sample by more
// than the float32 rounding of its position, and at steep yarn slopes and
// sharp specular lobes one ulp of position already changes a sample's
// integrand by up to 1e-3 relative.  The hardware approximations (v_sin,
// v_cos with their absolute error) are therefore not used on this path.
__device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
// The hardware reciprocal square root (1 ulp) for arguments >= 1, where the
// library's rsqrtf adds nothing but its rescaling of denormal inputs.
__device__ inline float rsqrt_ge1(float x) { return __builtin_amdgcn_rsqf(x); }
// The hardware square root (1 ulp) of a shading term 1 - a b with float32
// a, b in [0, 1] (0 or at least 2^-48, never denormal), in place of the
// library's correctly rounded sqrtf with its rescaling and correction steps.
__device__ inline float sqrt_term(float x) { return __builtin_amdgcn_sqrtf(x); }

// The two functions below replace the general library routines on the
// bounded arguments this model takes: polynomials in s = x^2 fitted to the
// functions on those intervals (least squares iteratively reweighted towards
// the minimax fit, coefficients rounded to float32; fit_model_polys.py
// beside this file derives them).  In float32 arithmetic they stay within 2
// ulp (sin pi x, cos pi x on |x| <= 1/4) and 4 ulp (tan x on |x| <= 1.5) of
// the exact functions, without the library's argument reduction and its
// branches.

// sin(pi x) = x S(s) and cos(pi x) = 1 + s C(s) for |x| <= 1/4.
__device__ inline void sincospi_quarter(float x, float *sn, float *cs)
{
    const float s = x * x;
    float p = fmaf(s, -0.5890786647796631f, 2.549767255783081f);
    p = fmaf(p, s, -5.167707920074463f);
    p = fmaf(p, s, 3.1415927410125732f);
    float c = fmaf(s, 0.23212634027004242f, -1.3351378440856934f);
    c = fmaf(c, s, 4.05871057510376f);
    c = fmaf(c, s, -4.934802055358887f);
    *sn = x * p;
    *cs = fmaf(c, s, 1.0f);
}

// tan(x) for |x| <= 1.5 rad (cos x >= 0.07): tan x = x + x s Q(s) / d with
// the pole factored out, d = (pi/2)^2 - s (one rounding of the exact x^2
// against the constant's float32 head, then its tail), and Q fitted to
// ((pi/2)^2 - s) (tan(x)/x - 1) / s; the quotient is the rounded product by
// the reciprocal with one correction step.
__device__ inline float tan_small(float x)
{
    constexpr float kHalfPiSqHi = 2.4674010276794434f;     // (pi/2)^2 = hi + lo
    constexpr float kHalfPiSqLo = 7.259289702687965e-08f;
    const float s = x * x;
    float p = fmaf(s, -4.3158843254786916e-07f, -7.24434403309715e-06f);
    p = fmaf(p, s, -0.0001721783191896975f);
    p = fmaf(p, s, -0.004346469882875681f);
    p = fmaf(p, s, 0.822467029094696f);
    const float d = fmaf(-x, x, kHalfPiSqHi) + kHalfPiSqLo;
    const float num = (x * s) * p;
    const float r = rcp(d);
    float q = num * r;
    q = fmaf(fmaf(-d, q, num), r, q);
    return q + x;
}

// Shirley-Chiu concentric mapping of [0,1)^2 onto the unit disk; the angle
// is pi/4 (b/a) or pi/2 - pi/4 (a/b): sin and cos of pi (q/4), swapped in the
// second case.  q is the product by the hardware reciprocal of the larger
// coordinate with one correction step from the exact residual (within an ulp
// of the quotient, |q| <= 1; the larger coordinate is at least 2^-25 in
// magnitude, never denormal).
__device__ inline float2 concentric_disk(float x, float y)
{
    float a = 2.0f * x - 1.0f, b = 2.0f * y - 1.0f;
    if (a == 0.0f && b == 0.0f)
        return make_float2(0.0f, 0.0f);
    const bool horiz = fabsf(a) > fabsf(b);
    const float rad = horiz ? a : b, num = horiz ? b : a;
    const float rr = rcp(rad);
    float q = num * rr;
    q = fmaf(fmaf(-rad, q, num), rr, q);
    float sn, cs;
    sincospi_quarter(0.25f * q, &sn, &cs);
    return horiz ? make_float2(rad * cs, rad * sn) : make_float2(rad * sn, rad * cs);
}

// x reduced into [0, period) (period a small positive integer as float).
__device__ inline float wrap_period(float x, float period, float inv_period)
{
    float r = x - period * floorf(x * inv_period);
    r = r < 0.0f ? r + period : r;
    r = r >= period ? r - period : r;
    return r;
}

struct SampleVal {
    int yarn;       // kWarp, kWeft or kHole
    float num_c;    // rho_d * A: diffuse numerator of Eq. (3) per unit k_d
    float num_s;    // rho_s * A: specular numerator per unit k_s
    float area;     // projected area A(p, wo) of Eq. (4), V = 1
};

// The integrand of Eq. (3) and weight of Eq. (4) at surface point (us, vs).
// Texel column (or row) of reduced coordinate q, wrapped into [0, size).
// q lies within two cells of the period (size >= kVisRes), so two
// corrections each way suffice; the clamps keep any other value (a huge
// coordinate whose float32 reduction is inexact) inside the table.
__device__ inline int texel_of(float q, int size)
{
    int k = (int)floorf(fminf(fmaxf(q, -4.0f), 4096.0f) * (float)kVisRes);
    k = k < 0 ? k + size : k;
    k = k < 0 ? k + size : k;
    k = k >= size ? k - size : k;
    k = k >= size ? k - size : k;
    return min(max(k, 0), size - 1);
}

// texel_of for a march position: within two cells of the period by
// construction (texel centre plus at most kVisSteps steps of at most one
// texel), so the clamps are not needed.
__device__ inline int texel_near(float q, int size)
{
    int k = (int)floorf(q * (float)kVisRes);
    k = k < 0 ? k + size : k;
    k = k < 0 ? k + size : k;
    k = k >= size ? k - size : k;
    return k >= size ? k - size : k;
}

// V(x_p, w) of Eq. (3)-(4) for the point in texel (a0, b0), w.z > 0: a ray
// from the texel's centre at its height, one texel per step along the major
// horizontal axis of w (w_minor / |w_major| per texel along the other,
// rising w.z / |w_major| per texel), for at most kVisSteps steps; blocked
// where the texel under the ray is higher than the ray, free once the ray
// is above the highest texel.  Every position and ray height is float32
// with one rounding per operation (no contraction, correctly rounded
// division), so that each texel decision is reproducible.
__device__ inline bool vis_march(const float *__restrict__ tex, const VisFabric &vf, int a0,
                                 int b0, float3 w)
{
#pragma clang fp contract(off)
    const float inv_r = 1.0f / (float)kVisRes;
    const float ax = fabsf(w.x), ay = fabsf(w.y);
    const float major = ax >= ay ? ax : ay;
    if (!(major > 0.0f))
        return true;
    const float *t = tex + vf.off;
    const float h0 = t[b0 * vf.tw + a0];
    float du, dv;
    if (ax >= ay) {
        du = w.x > 0.0f ? inv_r : -inv_r;
        dv = (w.y / ax) * inv_r;
    } else {
        dv = w.y > 0.0f ? inv_r : -inv_r;
        du = (w.x / ay) * inv_r;
    }
    const float rise = (w.z / major) * inv_r;
    const float cu = ((float)a0 + 0.5f) * inv_r, cv = ((float)b0 + 0.5f) * inv_r;
    // Along the major axis the position is the texel centre +- k texels
    // exactly, so its texel index steps by one (wrapped); the minor axis
    // takes the rounded float32 position (|w_minor / w_major| <= 1, so it
    // moves at most one texel per step).  Table reads use 32-bit offsets.
    const bool major_u = ax >= ay;
    const int step = major_u ? (w.x > 0.0f ? 1 : -1) : (w.y > 0.0f ? 1 : -1);
    const int span = major_u ? vf.tw : vf.th;
    int m = major_u ? a0 : b0;
    for (int k = 1; k <= kVisSteps; k++) {
        const float fk = (float)k;
        const float h = h0 + fk * rise;
        if (h >= vf.hmax)
            return true;
        m += step;
        m = m == span ? 0 : (m < 0 ? span - 1 : m);
        const int a = major_u ? m : texel_near(cu + fk * du, vf.tw);
        const int b = major_u ? texel_near(cv + fk * dv, vf.th) : m;
        if (*(const float *)((const char *)t + (uint32_t)(b * vf.tw + a) * 4u) > h)
            return false;
    }
    return true;
}

// One footprint sample.  VIS: multiply A(p, wo) by V(x_p, wo) and the
// integrand by V(x_p, wi) (Eq. (3)-(4)); otherwise V = 1.
template <bool VIS>
__device__ inline SampleVal eval_surface_point(const DevFabric &f, float us, float vs,
                                               float3 wi, float3 wo, const float *tex,
                                               const VisFabric &vf)
{
    SampleVal out;
    float up = wrap_period(us, f.fwx, f.inv_wx);
    float vp = wrap_period(vs, f.fwy, f.inv_wy);
    int ta = 0, tb = 0;
    bool vis_o = true;
    if (VIS) {
        ta = texel_of(up, vf.tw);
        tb = texel_of(vp, vf.th);
        vis_o = vis_march(tex, vf, ta, tb, wo);
    }
    // Clamped so that even a huge finite uv, whose FP32 reduction is inexact,
    // indexes inside the cell table.
    int i = min(max((int)up, 0), f.wx - 1);
    int j = min(max((int)vp, 0), f.wy - 1);
    float s = up - (float)i, t = vp - (float)j;

    bool cov_warp = fabsf(s - 0.5f) <= f.half_width[0];
    bool cov_weft = fabsf(t - 0.5f) <= f.half_width[1];
    uint32_t cell = f.cell[j * 16 + i];
    bool warp_top = (cell >> 15) != 0;
    int yarn;
    if (warp_top)
        yarn = cov_warp ? kWarp : (cov_weft ? kWeft : kHole);
    else
        yarn = cov_weft ? kWeft : (cov_warp ? kWarp : kHole);
    out.yarn = yarn;
    if (yarn == kHole) {
        // The gap between yarns: nothing reflects, the macro plane projects wo.z.
        out.num_c = 0.0f;
        out.num_s = 0.0f;
        out.area = vis_o ? wo.z : 0.0f;
        return out;
    }
    const int y = yarn;
    const bool is_warp = y == kWarp;
    bool on_top = is_warp == warp_top;

    // Position across the yarn in [-1, 1] and along its float in [-1, 1).
    float across = ((is_warp ? s : t) - 0.5f) * f.inv_half_width[y];
    float along = 0.0f;
    uint32_t len = (cell >> 5) & 31u;
    if (on_top && len != 0u) {
        float off = (float)(cell & 31u);
        along = 2.0f * (off + (is_warp ? t : s)) * rcp((float)len) - 1.0f;
    }
    // |incl * along| <= pi/2 * 1 and |theta_max * across| <= pi/3 (inclination
    // is validated to at most 1.5 rad, |along|, |across| <= 1).
    float ma = f.beta[y] * tan_small(f.incl[y] * along);
    float mb = f.beta[y] * tan_small(kThetaMax * across);

    // Height-field normal m = (slopes, 1); n_p = m / |m|, n_p.z = 1/|m|.
    float mx = is_warp ? mb : ma, my = is_warp ? ma : mb;
    float len2 = 1.0f + ma * ma + mb * mb;
    float rl = rsqrt_ge1(len2);
    float jac = len2 * rl;                       // 1 / <n_s . n_p>
    float3 n = make_float3(mx * rl, my * rl, rl);
    // Yarn axis t0 (tilted with the float) and its twist about n_p.
    float re = rsqrt_ge1(1.0f + ma * ma);
    float3 t0 = is_warp ? make_float3(0.0f, re, -ma * re) : make_float3(re, 0.0f, -ma * re);
    float3 bx = make_float3(n.y * t0.z - n.z * t0.y, n.z * t0.x - n.x * t0.z,
                            n.x * t0.y - n.y * t0.x);
    float ct = f.cos_twist[y], st = f.sin_twist[y];
    float3 tp = make_float3(ct * t0.x + st * bx.x, ct * t0.y + st * bx.y, ct * t0.z + st * bx.z);

    float ci = wi.x * n.x + wi.y * n.y + wi.z * n.z;
    float co = wo.x * n.x + wo.y * n.y + wo.z * n.z;
    out.area = vis_o ? fmaxf(co, 0.0f) * jac : 0.0f;
    // Light below the fabric is transmitted (it must reach the ply from
    // below too); light above is reflected (from above the ply).  Light from
    // below is not shadowed by the height field.
    const bool transmit = wi.z < 0.0f;
    const bool lit = transmit ? ci < 0.0f : ci > 0.0f;
    if (!(lit && co > 0.0f && vis_o) || (VIS && !transmit && !vis_march(tex, vf, ta, tb, wi))) {
        out.num_c = 0.0f;
        out.num_s = 0.0f;
        return out;
    }
    const float aci = fabsf(ci);
    // Specular: fiber SGGX with S = I - (1 - alpha^2) t t^T, so that
    // h^T S^-1 h = 1 + (1/alpha^2 - 1)(h.t)^2 and w^T S w = 1 - (1 - alpha^2)(w.t)^2.
    float hx = wi.x + wo.x, hy = wi.y + wo.y, hz = wi.z + wo.z;
    const float h2 = hx * hx + hy * hy + hz * hz;
    float hr = rsqrtf(h2);
    float ht = (hx * tp.x + hy * tp.y + hz * tp.z) * hr;
    float it = wi.x * tp.x + wi.y * tp.y + wi.z * tp.z;
    float ot = wo.x * tp.x + wo.y * tp.y + wo.z * tp.z;
    float q = 1.0f + f.ia2m1[y] * ht * ht;
    float D = f.inv_pi_alpha[y] * rcp(q * q);
    float sig_i = sqrt_term(fmaxf(1.0f - f.alpha2m1[y] * it * it, 0.0f));
    float sig_o = sqrt_term(fmaxf(1.0f - f.alpha2m1[y] * ot * ot, 0.0f));
    const float lam_i = sig_i * rcp(aci), lam_o = sig_o * rcp(co);
    float G;
    if (!transmit) {
        // L >= sigma_i + sigma_o >= 2 alpha, so 1 - e^{-2L} loses at most a
        // few ulps to cancellation for the roughness range of fabrics.
        const float L = lam_i + lam_o;
        G = (1.0f - __expf(-kTRho * L)) * rcp(L);
    } else {
        // Single scattering between the slab's faces:
        // (e^{-T Lo} - e^{-T Li}) / (Li - Lo) = e^{-T m} (1 - e^{-T d}) / d
        // with m = min(Li, Lo) and d = |Li - Lo| (no overflow for either
        // order), 1 - e^{-T d} by expm1 so that it stays accurate (and the
        // quotient tends to T) as d -> 0.  Straight-through light has no flake.
        const float d = fabsf(lam_i - lam_o);
        const float frac = d > 0.0f ? -expm1f(-kTRho * d) / d : kTRho;
        G = h2 > 1e-18f ? __expf(-kTRho * fminf(lam_i, lam_o)) * frac : 0.0f;
    }
    // rho_s * A = D G / (4 |ci| co) * |ci| * co * jac
    out.num_s = 0.25f * D * G * jac;
    // Blended Lambertian of Eq. (1) per unit k_d, times <wi.n_p> and A; in
    // transmission its Lambertian share (1 - w)/pi.
    float w = f.wblend[y];
    float fd = (transmit ? (1.0f - w) : (w * ci * rcp(wi.z) + (1.0f - w))) * (1.0f / kPi);
    out.num_c = fd * aci * out.area;
    return out;
}

// Footprint sample in stratum (kx, ky) of a side x side grid, jittered by the
// SplitMix64 draw z; position in cells.  The stratum coordinates are divided
// by side correctly rounded: POW2 (side a power of two) multiplies by the
// exact reciprocal, which gives the same quotient without a division.
template <bool POW2>
__device__ inline float2 footprint_sample(uint64_t z, int kx, int ky, float side, float u,
                                          float v, float r)
{
    const float x = (float)kx + u24_hi(z), y = (float)ky + u24_mid(z);
    const float inv = 1.0f / side;
    const float2 d = POW2 ? concentric_disk(x * inv, y * inv) : concentric_disk(x / side, y / side);
    return make_float2(fmaf(r, d.x, u), fmaf(r, d.y, v));
}
__host__ __device__ inline bool is_pow2(int side) { return side > 0 && (side & (side - 1)) == 0; }

// A pixel whose inputs fall outside the model's domain (shaded as 0).
__device__ inline bool pixel_fault(int fid, int n_fabrics, float u, float v, float r, float3 wi,
                                   float3 wo)
{
    bool finite = isfinite(u) && isfinite(v) && isfinite(r) && isfinite(wi.x) &&
                  isfinite(wi.y) && isfinite(wi.z) && isfinite(wo.x) && isfinite(wo.y) &&
                  isfinite(wo.z);
    return !finite || fid >= n_fabrics || !(r > 0.0f) || wi.z == 0.0f || !(wo.z > 0.0f);
}

// Wave-wide FP64 footprint estimate for one pixel: lanes take samples
// lane, lane + 64, ...; partial sums are reduced across the wave in a fixed
// butterfly order.  Every lane returns the four components.
template <bool VIS, bool POW2>
__device__ inline void filter_pixel_wave(const DevFabric &f, uint64_t seed, uint64_t pixel,
                                         int n_samples, int side, float u,
                                         float v, float r, float3 wi, float3 wo, int lane,
                                         const float *tex, const VisFabric &vf, double comp[4])
{
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    // Sample k = lane + 64 i draws output pixel * N + k of SplitMix64(seed):
    // the generator state advances by 64 gammas per iteration, and the
    // stratum (kx, ky) = (k mod side, k div side) by 64 with one carry.
    uint64_t state = seed + ((uint64_t)pixel * (uint64_t)n_samples + (uint64_t)lane + 1ull) * kGoldenGamma;
    const uint64_t step = 64ull * kGoldenGamma;
    const int dky = 64 / side, dkx = 64 - dky * side;
    int ky = lane / side, kx = lane - ky * side;
    for (int k = lane; k < n_samples; k += 64, state += step) {
        float2 pos = footprint_sample<POW2>(splitmix64_mix(state), kx, ky, (float)side, u, v, r);
        kx += dkx;
        ky += dky;
        if (kx >= side) {
            kx -= side;
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
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int c = 0; c < 5; c++)
            acc[c] += __shfl_xor(acc[c], off, 64);
    }
    for (int c = 0; c < 4; c++)
        comp[c] = acc[4] > 0.0 ? acc[c] / acc[4] : 0.0;
}

}  // namespace fab
