/*
 * FP64 CPU oracle for footprint-filtered woven-fabric shading and its neural
 * decoder, after Chen, Wang and Wang, "Real-time Neural Woven Fabric
 * Rendering" (SIGGRAPH Conference Papers 2024).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no source,
 * header, table or constant generator with the HIP library, and the product
 * path never calls it.
 *
 * What it computes, in plain double precision and in the order the paper
 * states it:
 *   - the point shading model: Eq. (1) (specular SpongeCake layer with a
 *     fiber-like SGGX microflake plus the blended Lambertian term) with D, G
 *     and Lambda from Eq. (2), S = R^T diag(1,1,alpha^2) R and T*rho = 2
 *     (Sec. 3.1); for light from below the fabric (wi.z < 0) a transmission
 *     lobe: the single scattering of the same slab between its two faces
 *     (Wang et al. 2021), plus the Lambertian share (1 - w)/pi (the paper's
 *     BTDF is in its supplementary: "parity unpinned", pinned by
 *     reciprocity and energy bounds);
 *   - a procedural yarn geometry that yields the ply normal n_p and
 *     orientation t_p from the weave pattern and the per-yarn parameters of
 *     Table 1 (the paper takes it from Jin et al.; its exact form lives in the
 *     paper's supplementary, so this stand-in is "parity unpinned" against the
 *     paper's own geometry and pinned only by its invariants);
 *   - the footprint aggregation of Eq. (3) with A(p, wo) of Eq. (4) and the
 *     normaliser A_P of Eq. (5), estimated by stratified, jittered
 *     Monte-Carlo samples over a disk footprint, split into the four
 *     components of Eq. (7) whose albedo-weighted sum is Eq. (8); the binary
 *     visibility V of Eq. (3)-(4) is either 1 or the inter-yarn
 *     shadowing-masking of a stand-in height field (integrated from the same
 *     yarn slopes, tabulated per texel, marched over a fixed two-cell patch:
 *     the paper's own definition is in its supplementary, so this part is
 *     "parity unpinned" against the paper and pinned by its invariants);
 *   - the network of Sec. 4.2 at the sizes of this build (encoder: one-hot
 *     weave grid + 12 yarn scalars -> residual MLP -> latent 32; decoder:
 *     spatial fusion of latent and encoded footprint, then the angular
 *     decoder with wi.xyz and wo.xy), forward and backward;
 *   - the loss of Eq. (9)-(11) and an Adam step (Kingma and Ba 2015, Alg. 1);
 *   - the decoder at the paper's own form (latent 64, one-blob footprint
 *     encoding to 24 channels, two fusion layers, a five-layer angular
 *     decoder with one residual skip, leaky ReLU), forward only.
 *
 * Random numbers: the jitter of footprint samples and the training-batch
 * recipe draw from SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), written
 * here from its published definition.  Footprint disk samples use the
 * concentric square-to-disk map of Shirley and Chiu (1997).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.141592653589793238462643383279502884

/* Cross-section slope limit of the stand-in yarn profile (radians). */
#define ORC_THETA_MAX (ORC_PI / 3.0)
/* Optical depth T*rho of the specular layer, fixed to 2 for fabrics (Sec. 3.1). */
#define ORC_T_RHO 2.0
/* k of the specular log mapping g(x) = ln(k x + 1) (Eq. (9)): 100 for
 * reflection, 1000 for transmission (Sec. 4.2). */
#define ORC_K_SPEC 100.0
#define ORC_K_SPEC_T 1000.0
/* Loss weights lambda_S and lambda_C (Eq. (11)). */
#define ORC_LAMBDA_S 0.4
#define ORC_LAMBDA_C 0.1
/* A footprint sample this close (cells) to a classification edge is flagged. */
#define ORC_EDGE_EPS 1e-5
/* With visibility, a sample this close (cells) to a texel boundary is
 * flagged: float32 positions computed in another order may pick the
 * neighbouring texel as the ray's start. */
#define ORC_TEXEL_EPS 4e-6
/* Visibility: height-field texels per cell and axis, and march length in
 * texel steps along the direction's major horizontal axis (two cells). */
#define ORC_VIS_RES 16
#define ORC_VIS_STEPS 32

enum { ORC_WARP = 0, ORC_WEFT = 1, ORC_HOLE = 2 };

/* One fabric: weave pattern plus the Table 1 parameters per yarn type
 * (index 0 = warp, 1 = weft) and the albedos of Eq. (8). */
typedef struct {
    int32_t wx, wy;            /* pattern period in cells (columns, rows) */
    uint8_t pattern[256];      /* P[j][i] at pattern[j * wx + i]; 1 = warp on top */
    double alpha[2];           /* roughness */
    double beta[2];            /* height-field scaling */
    double twist[2];           /* twist angle psi (rad) */
    double incl[2];            /* inclination angle u (rad) */
    double gap[2];             /* gap fraction of the yarn width */
    double wblend[2];          /* diffuse blend weight w of Eq. (1) */
    double kd[2][3];           /* diffuse albedo RGB */
    double ks[2][3];           /* specular albedo RGB */
} orc_material;

/* ------------------------------------------------------------------------ */
/* Small vector helpers                                                      */
/* ------------------------------------------------------------------------ */

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static void cross3(const double a[3], const double b[3], double out[3])
{
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

static void normalize3(double a[3])
{
    double l = sqrt(dot3(a, a));
    a[0] /= l;
    a[1] /= l;
    a[2] /= l;
}

/* x mod period, in [0, period). */
static double floor_mod(double x, double period)
{
    double r = fmod(x, period);
    if (r < 0.0)
        r += period;
    if (r >= period)
        r -= period;
    return r;
}

static int imod(int a, int m)
{
    int r = a % m;
    return r < 0 ? r + m : r;
}

/* ------------------------------------------------------------------------ */
/* SplitMix64 and the concentric disk map                                   */
/* ------------------------------------------------------------------------ */

/* The index-th output (index 0 first) of a SplitMix64 generator whose state
 * starts at `seed`: the state advances by the golden-gamma constant, and each
 * output is the variant-13 mix of the new state. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t index)
{
    uint64_t z = seed + (index + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Two 24-bit uniforms in [0, 1) from one 64-bit output: bits 63..40 and 39..16. */
static void u24_pair(uint64_t z, double *a, double *b)
{
    *a = (double)(z >> 40) * (1.0 / 16777216.0);
    *b = (double)((z >> 16) & 0xFFFFFFull) * (1.0 / 16777216.0);
}

/* Shirley-Chiu concentric map of the unit square onto the unit disk. */
void orc_concentric(double x, double y, double out[2])
{
    double a = 2.0 * x - 1.0, b = 2.0 * y - 1.0;
    double rad, phi;
    if (a == 0.0 && b == 0.0) {
        out[0] = 0.0;
        out[1] = 0.0;
        return;
    }
    if (fabs(a) > fabs(b)) {
        rad = a;
        phi = (ORC_PI / 4.0) * (b / a);
    } else {
        rad = b;
        phi = ORC_PI / 2.0 - (ORC_PI / 4.0) * (a / b);
    }
    out[0] = rad * cos(phi);
    out[1] = rad * sin(phi);
}

/* ------------------------------------------------------------------------ */
/* Weave pattern and yarn geometry (Sec. 3.1, Table 1)                       */
/* ------------------------------------------------------------------------ */

static int pat(const orc_material *m, int i, int j)
{
    return m->pattern[j * m->wx + i] ? 1 : 0;
}

/* The warp run through cell (i, j): consecutive rows of column i (cyclic) in
 * which the warp is on top.  Returns 0 if the whole column is warp-on-top (no
 * interlacing, the yarn lies flat along its axis). */
static int warp_run(const orc_material *m, int i, int j, int *offset, int *length)
{
    int count = 0;
    for (int k = 0; k < m->wy; k++)
        count += pat(m, i, k);
    if (count == m->wy)
        return 0;
    int back = 0, fwd = 0;
    while (pat(m, i, imod(j - back - 1, m->wy)) == 1)
        back++;
    while (pat(m, i, imod(j + fwd + 1, m->wy)) == 1)
        fwd++;
    *offset = back;
    *length = back + fwd + 1;
    return 1;
}

/* The weft run through cell (i, j): consecutive columns of row j in which
 * the weft is on top. */
static int weft_run(const orc_material *m, int i, int j, int *offset, int *length)
{
    int count = 0;
    for (int k = 0; k < m->wx; k++)
        count += 1 - pat(m, k, j);
    if (count == m->wx)
        return 0;
    int back = 0, fwd = 0;
    while (pat(m, imod(i - back - 1, m->wx), j) == 0)
        back++;
    while (pat(m, imod(i + fwd + 1, m->wx), j) == 0)
        fwd++;
    *offset = back;
    *length = back + fwd + 1;
    return 1;
}

typedef struct {
    int yarn;          /* ORC_WARP, ORC_WEFT or ORC_HOLE */
    int on_top;        /* the visible yarn is the top yarn of its cell */
    int top;           /* the cell's top yarn type */
    double n[3];       /* ply normal n_p */
    double t[3];       /* ply orientation t_p */
    double edge;       /* distance (cells) to the nearest classification edge */
    double across;     /* across coordinate in [-1, 1] of the visible yarn */
    double along;      /* along coordinate in [-1, 1) (0 for a lower or flat yarn) */
    double run;        /* length (cells) of the float of a top yarn, 0 if flat */
    double up, vp;     /* the point reduced to the pattern period */
} orc_point;

/* Geometry at surface point (us, vs), in cells; the macro normal is +z, u
 * runs along +x (the weft direction) and v along +y (the warp direction). */
static void point_geometry(const orc_material *m, double us, double vs, orc_point *pt)
{
    double up = floor_mod(us, (double)m->wx);
    double vp = floor_mod(vs, (double)m->wy);
    int i = (int)floor(up), j = (int)floor(vp);
    if (i > m->wx - 1)
        i = m->wx - 1;
    if (j > m->wy - 1)
        j = m->wy - 1;
    double s = up - i, t = vp - j;
    pt->up = up;
    pt->vp = vp;
    pt->across = 0.0;
    pt->along = 0.0;
    pt->run = 0.0;

    /* A yarn covers the band of its cell outside the gap; both bounds inclusive. */
    double half_w = 0.5 * (1.0 - m->gap[ORC_WARP]);
    double half_f = 0.5 * (1.0 - m->gap[ORC_WEFT]);
    int cov_warp = fabs(s - 0.5) <= half_w;
    int cov_weft = fabs(t - 0.5) <= half_f;
    int warp_top = pat(m, i, j);
    pt->top = warp_top ? ORC_WARP : ORC_WEFT;

    double e = s;
    if (1.0 - s < e) e = 1.0 - s;
    if (t < e) e = t;
    if (1.0 - t < e) e = 1.0 - t;
    if (fabs(fabs(s - 0.5) - half_w) < e) e = fabs(fabs(s - 0.5) - half_w);
    if (fabs(fabs(t - 0.5) - half_f) < e) e = fabs(fabs(t - 0.5) - half_f);
    pt->edge = e;

    /* The top yarn wins where it covers; the lower yarn shows in its gap. */
    if (warp_top) {
        pt->yarn = cov_warp ? ORC_WARP : (cov_weft ? ORC_WEFT : ORC_HOLE);
        pt->on_top = pt->yarn == ORC_WARP;
    } else {
        pt->yarn = cov_weft ? ORC_WEFT : (cov_warp ? ORC_WARP : ORC_HOLE);
        pt->on_top = pt->yarn == ORC_WEFT;
    }
    if (pt->yarn == ORC_HOLE) {
        pt->n[0] = 0.0; pt->n[1] = 0.0; pt->n[2] = 1.0;
        pt->t[0] = 0.0; pt->t[1] = 0.0; pt->t[2] = 0.0;
        return;
    }

    int y = pt->yarn;
    /* across in [-1, 1] over the yarn's width; along in [-1, 1) over its float */
    double across = (y == ORC_WARP) ? (s - 0.5) / half_w : (t - 0.5) / half_f;
    double along = 0.0;
    if (pt->on_top) {
        int off, len, ok;
        if (y == ORC_WARP)
            ok = warp_run(m, i, j, &off, &len);
        else
            ok = weft_run(m, i, j, &off, &len);
        if (ok) {
            along = 2.0 * (off + (y == ORC_WARP ? t : s)) / len - 1.0;
            pt->run = len;
        }
    }
    pt->across = across;
    pt->along = along;

    /* Height-field slopes: the float arches along the yarn with the
     * inclination angle, the cross-section bulges with at most THETA_MAX;
     * beta scales both (it changes n_p and t_p, Sec. 3.1). */
    double ma = m->beta[y] * tan(m->incl[y] * along);
    double mb = m->beta[y] * tan(ORC_THETA_MAX * across);
    double d = sqrt(1.0 + ma * ma + mb * mb);
    double el = sqrt(1.0 + ma * ma);
    double t0[3];
    if (y == ORC_WARP) {
        pt->n[0] = mb / d; pt->n[1] = ma / d; pt->n[2] = 1.0 / d;
        t0[0] = 0.0; t0[1] = 1.0 / el; t0[2] = -ma / el;
    } else {
        pt->n[0] = ma / d; pt->n[1] = mb / d; pt->n[2] = 1.0 / d;
        t0[0] = 1.0 / el; t0[1] = 0.0; t0[2] = -ma / el;
    }
    /* Twist: rotate the yarn axis about n_p by psi (right-handed). */
    double b[3];
    cross3(pt->n, t0, b);
    double cp = cos(m->twist[y]), sp = sin(m->twist[y]);
    for (int k = 0; k < 3; k++)
        pt->t[k] = cp * t0[k] + sp * b[k];
}

/* ------------------------------------------------------------------------ */
/* Height field and inter-yarn visibility V of Eq. (3)-(4)                   */
/* ------------------------------------------------------------------------ */

/* Depth (cells) of a yarn's cap: the drop of its cross-section from the
 * crown (across = 0) to its edge (across = +-1). */
static double cap_depth(const orc_material *m, int y)
{
    double half = 0.5 * (1.0 - m->gap[y]);
    return m->beta[y] * half * (-log(cos(ORC_THETA_MAX))) / ORC_THETA_MAX;
}

/* Surface height (cells above the top yarns' crowns) at (us, vs): the
 * integral of the slopes that define n_p, so that the height field's
 * gradient is (-n_p.x, -n_p.y) / n_p.z.  Across a yarn the slope
 * beta tan(theta_max x') over the half-width integrates to
 * beta half / theta_max ln cos(theta_max x'); along a top yarn's float of
 * length L the slope beta tan(u y') integrates to
 * beta L / (2 u) ln cos(u y').  A lower yarn lies one cap depth of the top
 * yarn lower (its crown level with the top yarn's edges); a hole lies below
 * both caps. */
double orc_surface_height(const orc_material *m, double us, double vs)
{
    orc_point pt;
    point_geometry(m, us, vs, &pt);
    int top = pt.top, low = 1 - pt.top;
    if (pt.yarn == ORC_HOLE)
        return -cap_depth(m, top) - cap_depth(m, low);
    int y = pt.yarn;
    double half = 0.5 * (1.0 - m->gap[y]);
    double h = m->beta[y] * half / ORC_THETA_MAX * log(cos(ORC_THETA_MAX * pt.across));
    if (pt.on_top) {
        /* At zero inclination the float is flat: its term's limit is 0. */
        if (pt.run > 0.0 && m->incl[y] != 0.0)
            h += m->beta[y] * pt.run / (2.0 * m->incl[y]) * log(cos(m->incl[y] * pt.along));
    } else {
        h -= cap_depth(m, top);
    }
    return h;
}

/* The tabulated height field: texel (a, b) of the period, a < wx R, b < wy R,
 * holds the surface height at its centre rounded to float32.  Returns the
 * largest texel. */
float orc_height_table(const orc_material *m, float *table)
{
    int tw = m->wx * ORC_VIS_RES, th = m->wy * ORC_VIS_RES;
    float hmax = -INFINITY;
    for (int b = 0; b < th; b++)
        for (int a = 0; a < tw; a++) {
            float h = (float)orc_surface_height(m, (a + 0.5) / ORC_VIS_RES, (b + 0.5) / ORC_VIS_RES);
            table[b * tw + a] = h;
            if (h > hmax)
                hmax = h;
        }
    return hmax;
}

static int texel_wrap(float q, int size)
{
    int k = (int)floorf(q * (float)ORC_VIS_RES) % size;
    return k < 0 ? k + size : k;
}

/* V(x_p, w): 1 if a ray from the surface point toward w (w.z > 0) clears
 * the height field.  The ray leaves the centre of the point's texel at that
 * texel's height and advances one texel (1/R cell) per step along the major
 * horizontal axis of w and w_minor / |w_major| / R along the other, rising
 * w.z / |w_major| / R, for up to ORC_VIS_STEPS steps (a fixed two-cell
 * patch); it is blocked where the texel under it is higher than the ray,
 * and free once the ray is above the highest texel.  The positions and ray
 * heights are float32 arithmetic, one rounding per operation in the order
 * written, so that every texel decision is that of float32 (up, vp: the
 * point reduced to the period, as float32). */
int orc_visible(const float *table, int tw, int th, float hmax, float up, float vp,
                const double w[3])
{
    const float inv_r = 1.0f / (float)ORC_VIS_RES;
    float wx = (float)w[0], wy = (float)w[1], wz = (float)w[2];
    float ax = fabsf(wx), ay = fabsf(wy);
    float major = ax >= ay ? ax : ay;
    if (!(major > 0.0f))
        return 1;
    int a0 = texel_wrap(up, tw), b0 = texel_wrap(vp, th);
    float h0 = table[b0 * tw + a0];
    float cu = ((float)a0 + 0.5f) * inv_r, cv = ((float)b0 + 0.5f) * inv_r;
    float du, dv;
    if (ax >= ay) {
        du = wx > 0.0f ? inv_r : -inv_r;
        dv = (wy / ax) * inv_r;
    } else {
        dv = wy > 0.0f ? inv_r : -inv_r;
        du = (wx / ay) * inv_r;
    }
    float rise = (wz / major) * inv_r;
    for (int k = 1; k <= ORC_VIS_STEPS; k++) {
        float fk = (float)k;
        float prod = fk * rise;
        float h = h0 + prod;
        if (h >= hmax)
            return 1;
        float pu = fk * du, pv = fk * dv;
        float qu = cu + pu, qv = cv + pv;
        if (table[texel_wrap(qv, th) * tw + texel_wrap(qu, tw)] > h)
            return 0;
    }
    return 1;
}

/* V at (us, vs) for one material, building its table (test entry point). */
int orc_visible_at(const orc_material *m, double us, double vs, const double w[3])
{
    int tw = m->wx * ORC_VIS_RES, th = m->wy * ORC_VIS_RES;
    float *table = (float *)malloc(sizeof(float) * tw * th);
    float hmax = orc_height_table(m, table);
    orc_point pt;
    point_geometry(m, us, vs, &pt);
    int v = orc_visible(table, tw, th, hmax, (float)pt.up, (float)pt.vp, w);
    free(table);
    return v;
}

/* The height table of a material when visibility is on (NULL when off). */
typedef struct {
    const float *table;
    int tw, th;
    float hmax;
} orc_vis;

/* ------------------------------------------------------------------------ */
/* Point shading model, Eq. (1)-(2)                                          */
/* ------------------------------------------------------------------------ */

/* The SGGX matrix of a fiber-like microflake along t: S = R^T diag(1,1,a^2) R
 * where the rows of R are an orthonormal frame whose last axis is t. */
static void sggx_matrix(double alpha, const double t[3], double S[3][3])
{
    double e3[3] = {t[0], t[1], t[2]};
    normalize3(e3);
    double helper[3] = {1.0, 0.0, 0.0};
    if (fabs(e3[0]) > 0.9) {
        helper[0] = 0.0;
        helper[1] = 1.0;
    }
    double e1[3], e2[3];
    cross3(helper, e3, e1);
    normalize3(e1);
    cross3(e3, e1, e2);
    const double *R[3] = {e1, e2, e3};
    double diag[3] = {1.0, 1.0, alpha * alpha};
    for (int a = 0; a < 3; a++)
        for (int c = 0; c < 3; c++) {
            double acc = 0.0;
            for (int k = 0; k < 3; k++)
                acc += R[k][a] * diag[k] * R[k][c];
            S[a][c] = acc;
        }
}

static void inverse3(const double A[3][3], double inv[3][3])
{
    double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1])
               - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0])
               + A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    inv[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / det;
    inv[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det;
    inv[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det;
    inv[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / det;
    inv[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det;
    inv[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det;
    inv[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / det;
    inv[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det;
    inv[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det;
}

static double quad_form(const double M[3][3], const double w[3])
{
    double acc = 0.0;
    for (int a = 0; a < 3; a++)
        for (int c = 0; c < 3; c++)
            acc += w[a] * M[a][c] * w[c];
    return acc;
}

/* D(h) = 1 / (pi alpha q^2), q = h^T S^-1 h (Eq. (2)). */
double orc_sggx_D(double alpha, const double t[3], const double h[3])
{
    double S[3][3], Si[3][3];
    sggx_matrix(alpha, t, S);
    inverse3(S, Si);
    double q = quad_form(Si, h);
    return 1.0 / (ORC_PI * alpha * q * q);
}

/* sigma(w) = sqrt(w^T S w), the projected area (Eq. (2)). */
double orc_sggx_sigma(double alpha, const double t[3], const double w[3])
{
    double S[3][3];
    sggx_matrix(alpha, t, S);
    return sqrt(quad_form(S, w));
}

/* Transmission through the specular layer (light below the fabric,
 * wi.z < 0, and below the ply, ci < 0; viewer above both): single
 * scattering by the microflakes of a slab of optical depth T rho between its
 * faces.  A flake at depth d (from the top) scatters wi into wo with phase
 * D(h) / (4 sigma(wi)), h = (wi + wo)/|wi + wo|; the light reaching it is
 * attenuated by e^{-Lambda_i (T - d)}, the scattered light by
 * e^{-Lambda_o d}; integrating over d gives
 *   f_t = D / (4 |ci| co) (e^{-T Lambda_o} - e^{-T Lambda_i}) / (Lambda_i - Lambda_o)
 * (T e^{-T Lambda} when the two are equal), with Lambda(w) = sigma(w) / |w.n|.
 * The diffuse share is the Lambertian (1 - w)/pi.  Straight-through light
 * (wi = -wo, the excluded delta transmission) has no flake to scatter it. */
static void point_btdf(double alpha, double w, const double n[3], const double t[3],
                       const double wi[3], const double wo[3], double ci, double co, double out[2])
{
    double h[3] = {wi[0] + wo[0], wi[1] + wo[1], wi[2] + wo[2]};
    double hl = sqrt(dot3(h, h));
    out[1] = (1.0 - w) / ORC_PI;
    if (hl < 1e-9) {
        out[0] = 0.0;
        return;
    }
    for (int k = 0; k < 3; k++)
        h[k] /= hl;
    double D = orc_sggx_D(alpha, t, h);
    double lam_i = orc_sggx_sigma(alpha, t, wi) / -ci;
    double lam_o = orc_sggx_sigma(alpha, t, wo) / co;
    double d = lam_i - lam_o;
    double g = d != 0.0 ? (exp(-ORC_T_RHO * lam_o) - exp(-ORC_T_RHO * lam_i)) / d
                        : ORC_T_RHO * exp(-ORC_T_RHO * lam_o);
    out[0] = D * g / (4.0 * -ci * co);
}

/* f_s / k_s and f_d / k_d of Eq. (1) at a ply with normal n and orientation t.
 * Cosines are taken against the ply normal.  Reflection needs wi above the
 * macro surface and the ply, transmission wi below both; wo is always above
 * the ply; otherwise both lobes vanish.  wi[2] is the cosine against the
 * macro normal. */
void orc_point_brdf(double alpha, double w, const double n[3], const double t[3],
                    const double wi[3], const double wo[3], double out[2])
{
    double ci = dot3(wi, n), co = dot3(wo, n);
    if (co > 0.0 && ci < 0.0 && wi[2] < 0.0) {
        point_btdf(alpha, w, n, t, wi, wo, ci, co, out);
        return;
    }
    if (ci <= 0.0 || co <= 0.0 || wi[2] <= 0.0) {
        out[0] = 0.0;
        out[1] = 0.0;
        return;
    }
    double h[3] = {wi[0] + wo[0], wi[1] + wo[1], wi[2] + wo[2]};
    normalize3(h);
    double D = orc_sggx_D(alpha, t, h);
    double lam_i = orc_sggx_sigma(alpha, t, wi) / ci;   /* Lambda(wi) */
    double lam_o = orc_sggx_sigma(alpha, t, wo) / co;   /* Lambda(wo) */
    double L = lam_i + lam_o;
    double G = (1.0 - exp(-ORC_T_RHO * L)) / L;
    out[0] = D * G / (4.0 * ci * co);
    out[1] = w * ci / (ORC_PI * wi[2]) + (1.0 - w) / ORC_PI;
}

/* orc_point_brdf over n direction pairs wi[n][3], wo[n][3] at one ply; out[n][2]. */
void orc_point_brdf_batch(int64_t n, double alpha, double w, const double nrm[3], const double t[3],
                          const double *wi, const double *wo, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; k++)
        orc_point_brdf(alpha, w, nrm, t, wi + 3 * k, wo + 3 * k, out + 2 * k);
}

/* One footprint sample point: the visible yarn class, the two integrand
 * numerators of Eq. (3) per unit albedo (rho_S = f_s <wi.n_p>, rho_C =
 * f_d <wi.n_p>) and the projected-area weight A(p, wo) of Eq. (4).  A hole
 * is the empty macro surface: it reflects nothing and projects wo.z. */
typedef struct {
    orc_point geo;
    double rho_s, rho_c, area;
} orc_sample;

static void eval_point(const orc_material *m, const orc_vis *vis, double us, double vs,
                       const double wi[3], const double wo[3], orc_sample *smp)
{
    point_geometry(m, us, vs, &smp->geo);
    /* V(x_p, wo) enters A(p, wo) (Eq. (4)), V(x_p, wi) the integrand (Eq. (3)). */
    /* Light from below (transmission) is not shadowed by the height field. */
    double v_o = 1.0, v_i = 1.0;
    if (vis) {
        float up = (float)smp->geo.up, vp = (float)smp->geo.vp;
        v_o = orc_visible(vis->table, vis->tw, vis->th, vis->hmax, up, vp, wo);
        if (wi[2] > 0.0)
            v_i = orc_visible(vis->table, vis->tw, vis->th, vis->hmax, up, vp, wi);
    }
    if (smp->geo.yarn == ORC_HOLE) {
        smp->rho_s = 0.0;
        smp->rho_c = 0.0;
        smp->area = wo[2] * v_o;
        return;
    }
    int y = smp->geo.yarn;
    double f[2];
    orc_point_brdf(m->alpha[y], m->wblend[y], smp->geo.n, smp->geo.t, wi, wo, f);
    double ci = dot3(wi, smp->geo.n), co = dot3(wo, smp->geo.n);
    /* <wi.n_p> of Eq. (3): the cosine on the lit side of the ply (the lobes
     * are zero where wi and the ply disagree on the side). */
    double ci_lit = fabs(ci);
    smp->rho_s = f[0] * ci_lit * v_i;
    smp->rho_c = f[1] * ci_lit * v_i;
    /* <wo.n_p> / <n_s.n_p> V(x_p, wo); 1/<n_s.n_p> is the Jacobian. */
    smp->area = (co > 0.0 ? co : 0.0) / smp->geo.n[2] * v_o;
}

/* out[0..15]: yarn, on_top, edge, rho_s, rho_c, area, n[3], t[3], spare. */
void orc_point_eval(const orc_material *m, double us, double vs,
                    const double wi[3], const double wo[3], double out[16])
{
    orc_sample smp;
    eval_point(m, NULL, us, vs, wi, wo, &smp);
    memset(out, 0, 16 * sizeof(double));
    out[0] = smp.geo.yarn;
    out[1] = smp.geo.on_top;
    out[2] = smp.geo.edge;
    out[3] = smp.rho_s;
    out[4] = smp.rho_c;
    out[5] = smp.area;
    for (int k = 0; k < 3; k++) {
        out[6 + k] = smp.geo.n[k];
        out[9 + k] = smp.geo.t[k];
    }
}

/* orc_point_eval at n points (us[k], vs[k]) with fixed directions; out[n][16]. */
void orc_point_eval_batch(const orc_material *m, int64_t n, const double *us, const double *vs,
                          const double wi[3], const double wo[3], double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; k++)
        orc_point_eval(m, us[k], vs[k], wi, wo, out + 16 * k);
}

/* ------------------------------------------------------------------------ */
/* Footprint filter, Eq. (3)-(5), (7)                                        */
/* ------------------------------------------------------------------------ */

/* Footprint of radius r (cells) centred at (u, v) with a uniform disk kernel
 * k_P.  N = m*m stratified samples: stratum k = ky*m + kx is jittered by the
 * (pixel*N + k)-th SplitMix64 output of `seed` and mapped to the disk by the
 * concentric map.  The self-normalised estimate of Eq. (3)/(5) splits into
 * C_y = sum[yarn=y] rho_c A / sum A and S_y likewise (Eq. (7)); all four are 0
 * when sum A = 0.  With same_sample the sample uv is rounded to float32
 * before classification.  Returns the number of samples within
 * ORC_EDGE_EPS of a classification edge. */
static int filter_pixel(const orc_material *m, const orc_vis *vis, double u, double v,
                        double r, const double wi[3], const double wo[3], int n_samples,
                        uint64_t seed, uint64_t pixel, int same_sample, double comp[4],
                        double *area_sum)
{
    int side = (int)llround(sqrt((double)n_samples));
    double num[4] = {0.0, 0.0, 0.0, 0.0}, den = 0.0;
    int flagged = 0;
    for (int ky = 0; ky < side; ky++) {
        for (int kx = 0; kx < side; kx++) {
            uint64_t k = (uint64_t)ky * side + kx;
            double xi_x, xi_y, disk[2];
            u24_pair(orc_splitmix64(seed, pixel * (uint64_t)n_samples + k), &xi_x, &xi_y);
            orc_concentric((kx + xi_x) / side, (ky + xi_y) / side, disk);
            double us = u + r * disk[0];
            double vs = v + r * disk[1];
            if (same_sample) {
                us = (double)(float)us;
                vs = (double)(float)vs;
            }
            orc_sample smp;
            eval_point(m, vis, us, vs, wi, wo, &smp);
            int flag = smp.geo.edge < ORC_EDGE_EPS;
            if (vis) {
                double fu = smp.geo.up * ORC_VIS_RES, fv = smp.geo.vp * ORC_VIS_RES;
                double du = fu - floor(fu), dv = fv - floor(fv);
                if (fmin(du, 1.0 - du) < ORC_TEXEL_EPS * ORC_VIS_RES ||
                    fmin(dv, 1.0 - dv) < ORC_TEXEL_EPS * ORC_VIS_RES)
                    flag = 1;
            }
            flagged += flag;
            if (smp.geo.yarn != ORC_HOLE) {
                num[smp.geo.yarn] += smp.rho_c * smp.area;       /* C_warp, C_weft */
                num[2 + smp.geo.yarn] += smp.rho_s * smp.area;   /* S_warp, S_weft */
            }
            den += smp.area;
        }
    }
    for (int c = 0; c < 4; c++)
        comp[c] = den > 0.0 ? num[c] / den : 0.0;
    if (area_sum)
        *area_sum = den;
    return flagged;
}

/* Height tables of n materials (visibility on), or NULL arrays (off). */
static orc_vis *vis_tables(const orc_material *mats, int nmats, int visibility)
{
    if (!visibility)
        return NULL;
    orc_vis *vis = (orc_vis *)calloc(nmats, sizeof(orc_vis));
    for (int k = 0; k < nmats; k++) {
        vis[k].tw = mats[k].wx * ORC_VIS_RES;
        vis[k].th = mats[k].wy * ORC_VIS_RES;
        float *t = (float *)malloc(sizeof(float) * vis[k].tw * vis[k].th);
        vis[k].hmax = orc_height_table(&mats[k], t);
        vis[k].table = t;
    }
    return vis;
}

static void vis_free(orc_vis *vis, int nmats)
{
    if (!vis)
        return;
    for (int k = 0; k < nmats; k++)
        free((void *)vis[k].table);
    free(vis);
}

/* One pixel's filter; visibility != 0 includes V of Eq. (3)-(4). */
int orc_filter_pixel(const orc_material *m, double u, double v, double r,
                     const double wi[3], const double wo[3], int n_samples,
                     uint64_t seed, uint64_t pixel, int same_sample, int visibility,
                     double comp[4], double *area_sum)
{
    orc_vis *vis = vis_tables(m, 1, visibility);
    int fl = filter_pixel(m, vis, u, v, r, wi, wo, n_samples, seed, pixel, same_sample, comp,
                          area_sum);
    vis_free(vis, 1);
    return fl;
}

/* f_P = kd_warp C_warp + kd_weft C_weft + ks_warp S_warp + ks_weft S_weft (Eq. (8)). */
static void compose_rgb(const orc_material *m, const double comp[4], double rgb[3])
{
    for (int c = 0; c < 3; c++)
        rgb[c] = m->kd[0][c] * comp[0] + m->kd[1][c] * comp[1]
               + m->ks[0][c] * comp[2] + m->ks[1][c] * comp[3];
}

/* A pixel is a fault (all outputs 0) if any field is non-finite, the view is
 * not above the macro surface, the light grazes it exactly (wi.z = 0; below
 * it is transmission), the radius is not positive or the fabric id is out of
 * range. */
static int pixel_fault(int nmats, int fid, double u, double v, double r,
                       const double wi[3], const double wo[3])
{
    double f[9] = {u, v, r, wi[0], wi[1], wi[2], wo[0], wo[1], wo[2]};
    for (int k = 0; k < 9; k++)
        if (!isfinite(f[k]))
            return 1;
    if (fid < 0 || fid >= nmats || r <= 0.0 || wi[2] == 0.0 || wo[2] <= 0.0)
        return 1;
    return 0;
}

typedef struct {
    int64_t n;
    const uint16_t *fabric_id;
    const float *u, *v, *radius;
    const float *wi_x, *wi_y, *wi_z, *wo_x, *wo_y, *wo_z;
} orc_gbuffer;

static void load_pixel(const orc_gbuffer *g, int64_t p, int *fid, double *u, double *v,
                       double *r, double wi[3], double wo[3])
{
    *fid = g->fabric_id[p];
    *u = g->u[p];
    *v = g->v[p];
    *r = g->radius[p];
    wi[0] = g->wi_x[p]; wi[1] = g->wi_y[p]; wi[2] = g->wi_z[p];
    wo[0] = g->wo_x[p]; wo[1] = g->wo_y[p]; wo[2] = g->wo_z[p];
}

/* Filter every pixel of a G-buffer.  pixel_index[p] (or p if NULL) keys the
 * sample jitter.  comp is [4][n], rgb [3][n], flagged and fault [n]; any
 * output may be NULL.  Returns the number of faulted pixels. */
int64_t orc_filter_batch(const orc_material *mats, int nmats, const orc_gbuffer *g,
                         const int64_t *pixel_index, int n_samples, uint64_t seed,
                         int same_sample, int visibility, double *comp, double *rgb,
                         int32_t *flagged, int32_t *fault)
{
    int64_t n = g->n, faults = 0;
    orc_vis *vis = vis_tables(mats, nmats, visibility);
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : faults)
    for (int64_t p = 0; p < n; p++) {
        int fid;
        double u, v, r, wi[3], wo[3], c4[4] = {0, 0, 0, 0}, c3[3] = {0, 0, 0};
        load_pixel(g, p, &fid, &u, &v, &r, wi, wo);
        int bad = pixel_fault(nmats, fid, u, v, r, wi, wo);
        int fl = 0;
        if (!bad) {
            uint64_t key = pixel_index ? (uint64_t)pixel_index[p] : (uint64_t)p;
            fl = filter_pixel(&mats[fid], vis ? &vis[fid] : NULL, u, v, r, wi, wo, n_samples,
                              seed, key, same_sample, c4, NULL);
            compose_rgb(&mats[fid], c4, c3);
        }
        faults += bad;
        if (comp)
            for (int c = 0; c < 4; c++)
                comp[(int64_t)c * n + p] = c4[c];
        if (rgb)
            for (int c = 0; c < 3; c++)
                rgb[(int64_t)c * n + p] = c3[c];
        if (flagged)
            flagged[p] = fl;
        if (fault)
            fault[p] = bad;
    }
    vis_free(vis, nmats);
    return faults;
}

/* ------------------------------------------------------------------------ */
/* Network (Sec. 4.2)                                                        */
/* ------------------------------------------------------------------------ */

#define LATENT 32
#define NFEAT 40          /* 32 Fourier + 8 one-blob */
#define HID 64
#define NANG 5            /* wi.x, wi.y, wi.z, wo.x, wo.y */
#define NOUT 4            /* C_warp, C_weft, S_warp, S_weft */
#define X1 (LATENT + NFEAT)
#define X3 (HID + NANG)

/* Decoder parameter offsets (rows = output units, row-major). */
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + HID * X1)
#define OFF_W2 (OFF_B1 + HID)
#define OFF_B2 (OFF_W2 + HID * HID)
#define OFF_W3 (OFF_B2 + HID)
#define OFF_B3 (OFF_W3 + HID * X3)
#define OFF_W4 (OFF_B3 + HID)
#define OFF_B4 (OFF_W4 + NOUT * HID)
#define N_DEC (OFF_B4 + NOUT)

#define ENC_IN 524
#define ENC_HID 128
#define OFF_E1 0
#define OFF_C1 (OFF_E1 + ENC_HID * ENC_IN)
#define OFF_E2 (OFF_C1 + ENC_HID)
#define OFF_C2 (OFF_E2 + ENC_HID * ENC_HID)
#define OFF_E3 (OFF_C2 + ENC_HID)
#define OFF_C3 (OFF_E3 + ENC_HID * ENC_HID)
#define OFF_E4 (OFF_C3 + ENC_HID)
#define OFF_C4 (OFF_E4 + LATENT * ENC_HID)
#define N_ENC (OFF_C4 + LATENT)

int orc_param_counts(int out[2])
{
    out[0] = N_DEC;
    out[1] = N_ENC;
    return N_DEC + N_ENC;
}

static double relu(double x)
{
    return x > 0.0 ? x : 0.0;
}

static double frac(double x)
{
    return x - floor(x);
}

/* Spatial input of the decoder: the footprint position inside the pattern
 * period, p = (u mod Wx) / Wx and (v mod Wy) / Wy, as 8 Fourier frequencies
 * per axis, [sin 2 pi frac(2^k px), cos .., sin .. py, cos .. py] for
 * k = 0..7, followed by a one-blob encoding of the footprint size (Sec. 4.2):
 * tau = clamp((log2 r + 14) / 16, 0, 1) smeared over 8 Gaussian bins,
 * exp(-0.5 ((tau - (b + 1/2)/8) * 8)^2). */
void orc_spatial_features(double u, double v, double r, int wx, int wy, double s[NFEAT])
{
    double px = floor_mod(u, wx) / wx;
    double py = floor_mod(v, wy) / wy;
    for (int k = 0; k < 8; k++) {
        double f = (double)(1 << k);
        s[k] = sin(2.0 * ORC_PI * frac(f * px));
        s[8 + k] = cos(2.0 * ORC_PI * frac(f * px));
        s[16 + k] = sin(2.0 * ORC_PI * frac(f * py));
        s[24 + k] = cos(2.0 * ORC_PI * frac(f * py));
    }
    double tau = (log2(r) + 14.0) / 16.0;
    if (tau < 0.0) tau = 0.0;
    if (tau > 1.0) tau = 1.0;
    for (int b = 0; b < 8; b++) {
        double d = (tau - (b + 0.5) / 8.0) * 8.0;
        s[32 + b] = exp(-0.5 * d * d);
    }
}

/* y = W x + b for a row-major W[out][in]. */
static void dense(const double *W, const double *b, const double *x, int nin, int nout, double *y)
{
    for (int o = 0; o < nout; o++) {
        double acc = b[o];
        for (int i = 0; i < nin; i++)
            acc += W[o * nin + i] * x[i];
        y[o] = acc;
    }
}

/* Operand precision of the reduced-precision decoders (the rounding rule of
 * the reduced-precision paths: round to nearest, ties to even): x rounded to
 * `bits` significant bits within the format's exponent range; bits = 8 is
 * bfloat16 (binary32's exponent range), bits = 11 IEEE binary16 (spacing
 * 2^-24 below its smallest normal 2^-14, infinity beyond 65504 after
 * rounding).  bits <= 0 leaves x unchanged. */
double orc_round_operand(double x, int bits)
{
    if (bits <= 0 || x == 0.0 || !isfinite(x))
        return x;
    const int emin = bits == 11 ? -14 : -126;
    const double maxv = bits == 11 ? 65504.0 : 3.3895313892515355e38;
    int ex;
    frexp(x, &ex);                      /* |x| in [2^(ex-1), 2^ex) */
    int e = ex - 1;
    if (e < emin)
        e = emin;
    const double q = ldexp(1.0, e - (bits - 1));   /* the format's spacing at x */
    const double r = nearbyint(x / q) * q;         /* x / q is exact: q is 2^k */
    return fabs(r) > maxv ? copysign(INFINITY, x) : r;
}

/* dense() evaluated as a reduced-precision decoder evaluates it: each
 * product's two operands rounded to `bits` (orc_round_operand), except the
 * first `nfull` inputs and their weights (the latent, whose product the
 * decoders fold into the first layer's bias in full precision); bias and
 * sums exact. */
static void dense_q(const double *W, const double *b, const double *x, int nin, int nout,
                    int nfull, int bits, double *y)
{
    if (bits <= 0) {
        dense(W, b, x, nin, nout, y);
        return;
    }
    for (int o = 0; o < nout; o++) {
        double acc = b[o];
        for (int i = 0; i < nin; i++)
            acc += i < nfull ? W[o * nin + i] * x[i]
                             : orc_round_operand(W[o * nin + i], bits) * orc_round_operand(x[i], bits);
        y[o] = acc;
    }
}

/* Activations kept for the backward pass. */
typedef struct {
    double x1[X1], a1[HID], h1[HID], a2[HID], h2[HID], x3[X3], a3[HID], h3[HID], y[NOUT];
} dec_acts;

/* Decoder: spatial fusion h1 = relu(W1 [z, s] + b1), h2 = relu(W2 h1 + b2);
 * angular decoder h3 = relu(W3 [h2, wi.xyz, wo.xy] + b3), y = W4 h3 + b4.
 * bits > 0: products' operands rounded as in dense_q. */
static void decoder_forward(const double *P, const double *z, const double *s,
                            const double ang[NANG], int bits, dec_acts *A)
{
    for (int k = 0; k < LATENT; k++) A->x1[k] = z[k];
    for (int k = 0; k < NFEAT; k++) A->x1[LATENT + k] = s[k];
    dense_q(P + OFF_W1, P + OFF_B1, A->x1, X1, HID, LATENT, bits, A->a1);
    for (int k = 0; k < HID; k++) A->h1[k] = relu(A->a1[k]);
    dense_q(P + OFF_W2, P + OFF_B2, A->h1, HID, HID, 0, bits, A->a2);
    for (int k = 0; k < HID; k++) A->h2[k] = relu(A->a2[k]);
    for (int k = 0; k < HID; k++) A->x3[k] = A->h2[k];
    for (int k = 0; k < NANG; k++) A->x3[HID + k] = ang[k];
    dense_q(P + OFF_W3, P + OFF_B3, A->x3, X3, HID, 0, bits, A->a3);
    for (int k = 0; k < HID; k++) A->h3[k] = relu(A->a3[k]);
    dense_q(P + OFF_W4, P + OFF_B4, A->h3, HID, NOUT, 0, bits, A->y);
}

/* Accumulate dL/dW, dL/db for y = W x + b into G and return dL/dx in dx. */
static void dense_backward(const double *W, const double *x, const double *dy, int nin, int nout,
                           double *GW, double *Gb, double *dx)
{
    for (int i = 0; i < nin; i++)
        dx[i] = 0.0;
    for (int o = 0; o < nout; o++) {
        Gb[o] += dy[o];
        for (int i = 0; i < nin; i++) {
            GW[o * nin + i] += dy[o] * x[i];
            dx[i] += W[o * nin + i] * dy[o];
        }
    }
}

/* Backward through the decoder: adds parameter gradients into G and writes
 * dL/dz (the latent) into dz.  ReLU'(0) = 0. */
static void decoder_backward(const double *P, const dec_acts *A, const double dy[NOUT],
                             double *G, double dz[LATENT])
{
    double dh3[HID], da3[HID], dx3[X3], da2[HID], dh1[HID], da1[HID], dx1[X1];
    dense_backward(P + OFF_W4, A->h3, dy, HID, NOUT, G + OFF_W4, G + OFF_B4, dh3);
    for (int k = 0; k < HID; k++) da3[k] = A->a3[k] > 0.0 ? dh3[k] : 0.0;
    dense_backward(P + OFF_W3, A->x3, da3, X3, HID, G + OFF_W3, G + OFF_B3, dx3);
    for (int k = 0; k < HID; k++) da2[k] = A->a2[k] > 0.0 ? dx3[k] : 0.0;
    dense_backward(P + OFF_W2, A->h1, da2, HID, HID, G + OFF_W2, G + OFF_B2, dh1);
    for (int k = 0; k < HID; k++) da1[k] = A->a1[k] > 0.0 ? dh1[k] : 0.0;
    dense_backward(P + OFF_W1, A->x1, da1, X1, HID, G + OFF_W1, G + OFF_B1, dx1);
    for (int k = 0; k < LATENT; k++) dz[k] = dx1[k];
}

/* Components from the decoder's outputs: diffuse terms are linear, specular
 * terms invert the log mapping g of Eq. (9); both clamp at 0. */
/* k of Eq. (9) for a query: transmission when the light is below. */
static double spec_k(double wi_z) { return wi_z < 0.0 ? ORC_K_SPEC_T : ORC_K_SPEC; }

static void decode_outputs(const double y[NOUT], double k, double comp[4])
{
    comp[0] = relu(y[0]);
    comp[1] = relu(y[1]);
    comp[2] = relu((exp(y[2]) - 1.0) / k);
    comp[3] = relu((exp(y[3]) - 1.0) / k);
}

/* Decoder over a G-buffer with per-fabric latents z[nmats][32].  y is [4][n]
 * raw outputs, rgb [3][n] composed reflectance; faulted pixels give 0.
 * bits > 0: the decoder in that operand precision (dense_q). */
int64_t orc_decoder_batch_q(const double *P, const double *latents, const orc_material *mats,
                            int nmats, const orc_gbuffer *g, int bits, double *y, double *rgb)
{
    int64_t n = g->n, faults = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : faults)
    for (int64_t p = 0; p < n; p++) {
        int fid;
        double u, v, r, wi[3], wo[3], out[4] = {0, 0, 0, 0}, c3[3] = {0, 0, 0};
        load_pixel(g, p, &fid, &u, &v, &r, wi, wo);
        int bad = pixel_fault(nmats, fid, u, v, r, wi, wo);
        if (!bad) {
            double s[NFEAT], ang[NANG] = {wi[0], wi[1], wi[2], wo[0], wo[1]}, comp[4];
            dec_acts A;
            orc_spatial_features(u, v, r, mats[fid].wx, mats[fid].wy, s);
            decoder_forward(P, latents + (int64_t)fid * LATENT, s, ang, bits, &A);
            for (int c = 0; c < 4; c++) out[c] = A.y[c];
            decode_outputs(A.y, spec_k(wi[2]), comp);
            compose_rgb(&mats[fid], comp, c3);
        }
        faults += bad;
        if (y)
            for (int c = 0; c < 4; c++) y[(int64_t)c * n + p] = out[c];
        if (rgb)
            for (int c = 0; c < 3; c++) rgb[(int64_t)c * n + p] = c3[c];
    }
    return faults;
}

int64_t orc_decoder_batch(const double *P, const double *latents, const orc_material *mats,
                          int nmats, const orc_gbuffer *g, double *y, double *rgb)
{
    return orc_decoder_batch_q(P, latents, mats, nmats, g, 0, y, rgb);
}

/* ---- Paper-size decoder (Sec. 4.2 "Decoder", Fig. "network_whole") ------ */

/* One-blob encoding of the footprint (Sec. 4.2): 3 inputs to 24 channels,
 * 8 Gaussian bins (exp(-d^2/2), d in bins) each.  The position in the
 * pattern period, p = (u mod W_x)/W_x, is periodic, so its bins wrap: d is
 * the circular distance from 8p to the bin centre b + 1/2.  The size is
 * tau = clamp((log2 r + 14)/16, 0, 1) with ordinary bins.  Channels:
 * [u bins 0..7, v bins 0..7, size bins 0..7]. */
#define PBLOB 24
#define PLATENT 64
#define PHID 64
#define PX1 (PLATENT + PBLOB)
#define PXA1 (PHID + NANG)
#define P_WF1 0
#define P_BF1 (P_WF1 + PHID * PX1)
#define P_WF2 (P_BF1 + PHID)
#define P_BF2 (P_WF2 + PHID * PHID)
#define P_WA1 (P_BF2 + PHID)
#define P_BA1 (P_WA1 + PHID * PXA1)
#define P_WA2 (P_BA1 + PHID)
#define P_BA2 (P_WA2 + PHID * PHID)
#define P_WA3 (P_BA2 + PHID)
#define P_BA3 (P_WA3 + PHID * PHID)
#define P_WA4 (P_BA3 + PHID)
#define P_BA4 (P_WA4 + PHID * PHID)
#define P_WA5 (P_BA4 + PHID)
#define P_BA5 (P_WA5 + NOUT * PHID)
#define N_PDEC (P_BA5 + NOUT)
/* Leaky ReLU slope. */
#define ORC_LEAK 0.01

int orc_paper_param_count(void) { return N_PDEC; }

static double lrelu(double x) { return x > 0.0 ? x : ORC_LEAK * x; }

/* Footprint inputs without the encoding (the ablation of Sec. 5 "Encoding
 * of footprint"): the position fractions p_u, p_v and the size tau as plain
 * inputs, in the channels of their first one-blob bin (0, 8, 16); the other
 * channels are 0. */
void orc_paper_features_raw(double u, double v, double r, int wx, int wy, double f[PBLOB])
{
    for (int k = 0; k < PBLOB; k++) f[k] = 0.0;
    f[0] = floor_mod(u, wx) / wx;
    f[8] = floor_mod(v, wy) / wy;
    double tau = (log2(r) + 14.0) / 16.0;
    if (tau < 0.0) tau = 0.0;
    if (tau > 1.0) tau = 1.0;
    f[16] = tau;
}

void orc_paper_features(double u, double v, double r, int wx, int wy, double f[PBLOB])
{
    double p[2] = {floor_mod(u, wx) / wx, floor_mod(v, wy) / wy};
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 8; b++) {
            double d = 8.0 * p[a] - (b + 0.5);
            d -= 8.0 * floor((d + 4.0) / 8.0);     /* circular distance in [-4, 4) */
            f[8 * a + b] = exp(-0.5 * d * d);
        }
    double tau = (log2(r) + 14.0) / 16.0;
    if (tau < 0.0) tau = 0.0;
    if (tau > 1.0) tau = 1.0;
    for (int b = 0; b < 8; b++) {
        double d = 8.0 * tau - (b + 0.5);
        f[16 + b] = exp(-0.5 * d * d);
    }
}

/* Spatial fusion: two FC layers over [z, one-blob]; angular decoder: five
 * FC layers over [spatial feature, wi.xyz, wo.xy], the second and third a
 * residual block whose input is added before the block's last activation;
 * leaky ReLU after every layer but the output. */
/* Activations (after each leaky ReLU) kept for the backward pass. */
typedef struct {
    double x1[PX1], t[PHID], sp[PHID], xa[PXA1], x[PHID], h[PHID], rr[PHID], g[PHID], y[NOUT];
    double ang[NANG];
    int fused;
} paper_acts;

/* fused = 0: the network without the spatial fusion stage (the ablation of
 * Sec. 5 "Spatial fusion"): the angular inputs enter the first layer, through
 * A1's angular columns, and A1 sees zeros in their place; the parameter
 * layout and count are those of the paper's network. */
/* bits > 0: products' operands rounded as in dense_q (the residual add and
 * the activations exact). */
static void paper_forward_acts(const double *P, const double *z, const double f[PBLOB],
                               const double ang[NANG], int fused, int bits, paper_acts *A)
{
    for (int k = 0; k < PLATENT; k++) A->x1[k] = z[k];
    for (int k = 0; k < PBLOB; k++) A->x1[PLATENT + k] = f[k];
    for (int k = 0; k < NANG; k++) A->ang[k] = ang[k];
    A->fused = fused;
    dense_q(P + P_WF1, P + P_BF1, A->x1, PX1, PHID, PLATENT, bits, A->t);
    if (!fused)
        for (int o = 0; o < PHID; o++)
            for (int a = 0; a < NANG; a++)
                A->t[o] += orc_round_operand(P[P_WA1 + o * PXA1 + PHID + a], bits) *
                           orc_round_operand(ang[a], bits);
    for (int k = 0; k < PHID; k++) A->t[k] = lrelu(A->t[k]);
    dense_q(P + P_WF2, P + P_BF2, A->t, PHID, PHID, 0, bits, A->sp);
    for (int k = 0; k < PHID; k++) A->sp[k] = lrelu(A->sp[k]);
    for (int k = 0; k < PHID; k++) A->xa[k] = A->sp[k];
    for (int k = 0; k < NANG; k++) A->xa[PHID + k] = fused ? ang[k] : 0.0;
    dense_q(P + P_WA1, P + P_BA1, A->xa, PXA1, PHID, 0, bits, A->x);
    for (int k = 0; k < PHID; k++) A->x[k] = lrelu(A->x[k]);
    dense_q(P + P_WA2, P + P_BA2, A->x, PHID, PHID, 0, bits, A->h);
    for (int k = 0; k < PHID; k++) A->h[k] = lrelu(A->h[k]);
    dense_q(P + P_WA3, P + P_BA3, A->h, PHID, PHID, 0, bits, A->rr);
    for (int k = 0; k < PHID; k++) A->rr[k] = lrelu(A->rr[k] + A->x[k]);
    dense_q(P + P_WA4, P + P_BA4, A->rr, PHID, PHID, 0, bits, A->g);
    for (int k = 0; k < PHID; k++) A->g[k] = lrelu(A->g[k]);
    dense_q(P + P_WA5, P + P_BA5, A->g, PHID, NOUT, 0, bits, A->y);
}

static void paper_forward(const double *P, const double *z, const double f[PBLOB],
                          const double ang[NANG], int fused, int bits, double y[NOUT])
{
    paper_acts A;
    paper_forward_acts(P, z, f, ang, fused, bits, &A);
    for (int k = 0; k < NOUT; k++) y[k] = A.y[k];
}

/* Slope of the leaky ReLU at an activation a (its sign is the input's sign;
 * the slope at 0 is the leak). */
static double dlrelu(double a) { return a > 0.0 ? 1.0 : ORC_LEAK; }

/* Backward through the paper-size decoder: adds parameter gradients into G
 * and writes dL/dz into dz.  The residual block passes the gradient at A3's
 * activation input both through A3 and A2 and straight to A1's output. */
static void paper_backward(const double *P, const paper_acts *A, const double dy[NOUT],
                           double *G, double dz[PLATENT])
{
    double dg[PHID], drr[PHID], dh[PHID], dxb[PHID], dx[PHID], dxa[PXA1], dsp[PHID], dt[PHID];
    double dx1[PX1];
    dense_backward(P + P_WA5, A->g, dy, PHID, NOUT, G + P_WA5, G + P_BA5, dg);
    for (int k = 0; k < PHID; k++) dg[k] *= dlrelu(A->g[k]);
    dense_backward(P + P_WA4, A->rr, dg, PHID, PHID, G + P_WA4, G + P_BA4, drr);
    for (int k = 0; k < PHID; k++) drr[k] *= dlrelu(A->rr[k]);
    dense_backward(P + P_WA3, A->h, drr, PHID, PHID, G + P_WA3, G + P_BA3, dh);
    for (int k = 0; k < PHID; k++) dh[k] *= dlrelu(A->h[k]);
    dense_backward(P + P_WA2, A->x, dh, PHID, PHID, G + P_WA2, G + P_BA2, dxb);
    for (int k = 0; k < PHID; k++) dx[k] = (dxb[k] + drr[k]) * dlrelu(A->x[k]);
    dense_backward(P + P_WA1, A->xa, dx, PXA1, PHID, G + P_WA1, G + P_BA1, dxa);
    for (int k = 0; k < PHID; k++) dsp[k] = dxa[k] * dlrelu(A->sp[k]);
    dense_backward(P + P_WF2, A->t, dsp, PHID, PHID, G + P_WF2, G + P_BF2, dt);
    for (int k = 0; k < PHID; k++) dt[k] *= dlrelu(A->t[k]);
    if (!A->fused)     /* A1's angular columns act in the first layer */
        for (int o = 0; o < PHID; o++)
            for (int a = 0; a < NANG; a++)
                G[P_WA1 + o * PXA1 + PHID + a] += dt[o] * A->ang[a];
    dense_backward(P + P_WF1, A->x1, dt, PX1, PHID, G + P_WF1, G + P_BF1, dx1);
    for (int k = 0; k < PLATENT; k++) dz[k] = dx1[k];
}

/* The paper-size decoder over a G-buffer with per-fabric latents
 * z[nmats][64]: raw outputs y [4][n] and composed rgb [3][n] (decoded and
 * composed as the shading path does); faulted pixels give 0.  raw != 0:
 * footprint inputs without the one-blob encoding. */
int64_t orc_paper_decoder_batch_q(const double *P, const double *latents, const orc_material *mats,
                                  int nmats, const orc_gbuffer *g, int raw, int fused, int bits,
                                  double *y, double *rgb)
{
    int64_t n = g->n, faults = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : faults)
    for (int64_t p = 0; p < n; p++) {
        int fid;
        double u, v, r, wi[3], wo[3], out[4] = {0, 0, 0, 0}, c3[3] = {0, 0, 0};
        load_pixel(g, p, &fid, &u, &v, &r, wi, wo);
        int bad = pixel_fault(nmats, fid, u, v, r, wi, wo);
        if (!bad) {
            double f[PBLOB], ang[NANG] = {wi[0], wi[1], wi[2], wo[0], wo[1]}, comp[4];
            (raw ? orc_paper_features_raw : orc_paper_features)(u, v, r, mats[fid].wx, mats[fid].wy, f);
            paper_forward(P, latents + (int64_t)fid * PLATENT, f, ang, fused, bits, out);
            decode_outputs(out, spec_k(wi[2]), comp);
            compose_rgb(&mats[fid], comp, c3);
        }
        faults += bad;
        if (y)
            for (int c = 0; c < 4; c++) y[(int64_t)c * n + p] = out[c];
        if (rgb)
            for (int c = 0; c < 3; c++) rgb[(int64_t)c * n + p] = c3[c];
    }
    return faults;
}

int64_t orc_paper_decoder_batch(const double *P, const double *latents, const orc_material *mats,
                                int nmats, const orc_gbuffer *g, int raw, int fused, double *y,
                                double *rgb)
{
    return orc_paper_decoder_batch_q(P, latents, mats, nmats, g, raw, fused, 0, y, rgb);
}

/* ---- Encoder ------------------------------------------------------------ */

/* Fixed normalisation ranges of the 12 yarn scalars, ordered
 * [alpha_w, alpha_f, beta_w, beta_f, psi_w, psi_f, u_w, u_f, g_w, g_f, w_w, w_f]. */
static const double ENC_LO[6] = {0.1, 0.0, -ORC_PI / 6.0, ORC_PI / 12.0, 0.0, 0.0};
static const double ENC_HI[6] = {1.0, 2.0, ORC_PI / 6.0, ORC_PI / 4.0, 0.5, 1.0};

/* Encoder input: the weave as a 16 x 16 one-hot grid, cell (i, j) at
 * 2*(16 j + i) holding [P = 1, P = 0] inside the pattern and [0, 0] outside,
 * then the 12 yarn scalars min-max normalised. */
void orc_encoder_input(const orc_material *m, double x[ENC_IN])
{
    for (int k = 0; k < ENC_IN; k++)
        x[k] = 0.0;
    for (int j = 0; j < 16; j++)
        for (int i = 0; i < 16; i++)
            if (i < m->wx && j < m->wy) {
                int p = pat(m, i, j);
                x[2 * (16 * j + i) + 0] = p ? 1.0 : 0.0;
                x[2 * (16 * j + i) + 1] = p ? 0.0 : 1.0;
            }
    const double *vals[6] = {m->alpha, m->beta, m->twist, m->incl, m->gap, m->wblend};
    for (int q = 0; q < 6; q++)
        for (int y = 0; y < 2; y++)
            x[512 + 2 * q + y] = (vals[q][y] - ENC_LO[q]) / (ENC_HI[q] - ENC_LO[q]);
}

typedef struct {
    double x[ENC_IN], a1[ENC_HID], e1[ENC_HID], a2[ENC_HID], r2[ENC_HID], a3[ENC_HID],
        e2[ENC_HID], z[PLATENT];
} enc_acts;

/* The encoder's last layer for a latent of `lat` values: E4 [lat][128] at
 * OFF_E4, then c4 [lat]; the layers before it do not depend on lat. */
static int enc_off_c4(int lat) { return OFF_E4 + lat * ENC_HID; }

/* Encoder parameters for a latent of `lat` values (32: the config-size
 * network, 64: the paper-size network's encoder). */
int orc_encoder_param_count(int lat) { return enc_off_c4(lat) + lat; }

/* e1 = relu(E1 x + c1); residual block e2 = relu(e1 + E3 relu(E2 e1 + c2) + c3)
 * (two fully connected layers, skip added before the last activation, Sec. 4.2);
 * z = E4 e2 + c4 with `lat` outputs. */
static void encoder_forward_n(const double *Q, const orc_material *m, int lat, enc_acts *A)
{
    orc_encoder_input(m, A->x);
    dense(Q + OFF_E1, Q + OFF_C1, A->x, ENC_IN, ENC_HID, A->a1);
    for (int k = 0; k < ENC_HID; k++) A->e1[k] = relu(A->a1[k]);
    dense(Q + OFF_E2, Q + OFF_C2, A->e1, ENC_HID, ENC_HID, A->a2);
    for (int k = 0; k < ENC_HID; k++) A->r2[k] = relu(A->a2[k]);
    dense(Q + OFF_E3, Q + OFF_C3, A->r2, ENC_HID, ENC_HID, A->a3);
    for (int k = 0; k < ENC_HID; k++) A->a3[k] += A->e1[k];
    for (int k = 0; k < ENC_HID; k++) A->e2[k] = relu(A->a3[k]);
    dense(Q + OFF_E4, Q + enc_off_c4(lat), A->e2, ENC_HID, lat, A->z);
}

static void encoder_forward(const double *Q, const orc_material *m, enc_acts *A)
{
    encoder_forward_n(Q, m, LATENT, A);
}

static void encoder_backward_n(const double *Q, const enc_acts *A, const double *dz, int lat,
                               double *G)
{
    double de2[ENC_HID], da3[ENC_HID], dr2[ENC_HID], da2[ENC_HID], de1[ENC_HID], da1[ENC_HID],
        dx[ENC_IN];
    dense_backward(Q + OFF_E4, A->e2, dz, ENC_HID, lat, G + OFF_E4, G + enc_off_c4(lat), de2);
    for (int k = 0; k < ENC_HID; k++) da3[k] = A->a3[k] > 0.0 ? de2[k] : 0.0;
    dense_backward(Q + OFF_E3, A->r2, da3, ENC_HID, ENC_HID, G + OFF_E3, G + OFF_C3, dr2);
    for (int k = 0; k < ENC_HID; k++) da2[k] = A->a2[k] > 0.0 ? dr2[k] : 0.0;
    dense_backward(Q + OFF_E2, A->e1, da2, ENC_HID, ENC_HID, G + OFF_E2, G + OFF_C2, de1);
    for (int k = 0; k < ENC_HID; k++) de1[k] += da3[k];   /* skip connection */
    for (int k = 0; k < ENC_HID; k++) da1[k] = A->a1[k] > 0.0 ? de1[k] : 0.0;
    dense_backward(Q + OFF_E1, A->x, da1, ENC_IN, ENC_HID, G + OFF_E1, G + OFF_C1, dx);
}

static void encoder_backward(const double *Q, const enc_acts *A, const double dz[LATENT], double *G)
{
    encoder_backward_n(Q, A, dz, LATENT, G);
}

/* z[nmats][lat] from the encoder parameters Q of a latent of lat values. */
void orc_encoder_batch_n(const double *Q, const orc_material *mats, int nmats, int lat, double *z)
{
    for (int f = 0; f < nmats; f++) {
        enc_acts A;
        encoder_forward_n(Q, &mats[f], lat, &A);
        for (int k = 0; k < lat; k++)
            z[f * lat + k] = A.z[k];
    }
}

/* z[nmats][32] from the encoder parameters Q. */
void orc_encoder_batch(const double *Q, const orc_material *mats, int nmats, double *z)
{
    orc_encoder_batch_n(Q, mats, nmats, LATENT, z);
}

/* Gradient of the encoder parameters (grad, overwritten) from the latents'
 * gradients dz[nmats][lat], summed over the fabrics in order. */
void orc_encoder_backward_batch(const double *Q, const orc_material *mats, int nmats, int lat,
                                const double *dz, double *grad)
{
    memset(grad, 0, sizeof(double) * orc_encoder_param_count(lat));
    for (int f = 0; f < nmats; f++) {
        enc_acts A;
        encoder_forward_n(Q, &mats[f], lat, &A);
        encoder_backward_n(Q, &A, dz + (size_t)f * lat, lat, grad);
    }
}

/* ---- Loss, Eq. (9)-(11) ------------------------------------------------- */

/* Per-sample loss terms and dL/dy for outputs y and targets (C_warp, C_weft,
 * S_warp, S_weft).  With n samples in the batch, the loss is
 * sum_y lambda_S mean (y_S - ln(k S + 1))^2 + lambda_C mean (y_C - C)^2. */
static double loss_terms(const double y[NOUT], const double tgt[4], double k, int64_t n,
                         double dy[NOUT])
{
    double l = 0.0;
    for (int c = 0; c < 2; c++) {
        double d = y[c] - tgt[c];
        l += ORC_LAMBDA_C * d * d / (double)n;
        dy[c] = ORC_LAMBDA_C * 2.0 * d / (double)n;
    }
    for (int c = 2; c < 4; c++) {
        double d = y[c] - log(k * tgt[c] + 1.0);
        l += ORC_LAMBDA_S * d * d / (double)n;
        dy[c] = ORC_LAMBDA_S * 2.0 * d / (double)n;
    }
    return l;
}

/* Full forward, loss and backward of encoder + decoder on a batch.
 * params = [decoder | encoder]; grad has the same layout.  targets is [4][n].
 * Samples with faulted inputs contribute nothing (but still count in n).
 * dlatent (may be NULL) receives dL/dz per fabric [nmats][32].  Returns the loss. */
double orc_loss_grad(const double *params, const orc_material *mats, int nmats,
                     const orc_gbuffer *g, const float *targets, double *grad, double *dlatent)
{
    const double *P = params, *Q = params + N_DEC;
    int64_t n = g->n;
    double *z = (double *)malloc(sizeof(double) * nmats * LATENT);
    enc_acts *EA = (enc_acts *)malloc(sizeof(enc_acts) * (nmats > 0 ? nmats : 1));
    for (int f = 0; f < nmats; f++) {
        encoder_forward(Q, &mats[f], &EA[f]);
        for (int k = 0; k < LATENT; k++)
            z[f * LATENT + k] = EA[f].z[k];
    }
    memset(grad, 0, sizeof(double) * (N_DEC + N_ENC));
    double *dz = (double *)calloc((size_t)nmats * LATENT, sizeof(double));
    double loss = 0.0;
#ifdef _OPENMP
    int nth = omp_get_max_threads();
#else
    int nth = 1;
#endif
    double *Gt = (double *)calloc((size_t)nth * N_DEC, sizeof(double));
    double *dzt = (double *)calloc((size_t)nth * nmats * LATENT, sizeof(double));
    double *lt = (double *)calloc((size_t)nth, sizeof(double));
#pragma omp parallel
    {
#ifdef _OPENMP
        int tid = omp_get_thread_num();
#else
        int tid = 0;
#endif
        double *G = Gt + (size_t)tid * N_DEC;
        double *dzl = dzt + (size_t)tid * nmats * LATENT;
#pragma omp for schedule(static)
        for (int64_t p = 0; p < n; p++) {
            int fid;
            double u, v, r, wi[3], wo[3];
            load_pixel(g, p, &fid, &u, &v, &r, wi, wo);
            if (pixel_fault(nmats, fid, u, v, r, wi, wo))
                continue;
            double s[NFEAT], ang[NANG] = {wi[0], wi[1], wi[2], wo[0], wo[1]};
            double tgt[4], dy[NOUT], dzp[LATENT];
            for (int c = 0; c < 4; c++)
                tgt[c] = targets[(int64_t)c * n + p];
            dec_acts A;
            orc_spatial_features(u, v, r, mats[fid].wx, mats[fid].wy, s);
            decoder_forward(P, z + fid * LATENT, s, ang, 0, &A);
            lt[tid] += loss_terms(A.y, tgt, spec_k(wi[2]), n, dy);
            decoder_backward(P, &A, dy, G, dzp);
            for (int k = 0; k < LATENT; k++)
                dzl[fid * LATENT + k] += dzp[k];
        }
    }
    /* Fixed-order reduction of the per-thread partials. */
    for (int t = 0; t < nth; t++) {
        loss += lt[t];
        for (int k = 0; k < N_DEC; k++)
            grad[k] += Gt[(size_t)t * N_DEC + k];
        for (int k = 0; k < nmats * LATENT; k++)
            dz[k] += dzt[(size_t)t * nmats * LATENT + k];
    }
    for (int f = 0; f < nmats; f++)
        encoder_backward(Q, &EA[f], dz + f * LATENT, grad + N_DEC);
    if (dlatent)
        memcpy(dlatent, dz, sizeof(double) * nmats * LATENT);
    free(Gt);
    free(dzt);
    free(lt);
    free(dz);
    free(EA);
    free(z);
    return loss;
}

/* Decoder-only backward for given latents: dL/dparams (decoder part) and
 * dL/dlatent from upstream gradients dy[4][n] of the raw outputs. */
void orc_decoder_backward_batch(const double *P, const double *latents, const orc_material *mats,
                                int nmats, const orc_gbuffer *g, const double *dy_all,
                                double *grad_dec, double *grad_latent)
{
    int64_t n = g->n;
    memset(grad_dec, 0, sizeof(double) * N_DEC);
    memset(grad_latent, 0, sizeof(double) * nmats * LATENT);
    for (int64_t p = 0; p < n; p++) {
        int fid;
        double u, v, r, wi[3], wo[3];
        load_pixel(g, p, &fid, &u, &v, &r, wi, wo);
        if (pixel_fault(nmats, fid, u, v, r, wi, wo))
            continue;
        double s[NFEAT], ang[NANG] = {wi[0], wi[1], wi[2], wo[0], wo[1]}, dy[NOUT], dzp[LATENT];
        for (int c = 0; c < 4; c++)
            dy[c] = dy_all[(int64_t)c * n + p];
        dec_acts A;
        orc_spatial_features(u, v, r, mats[fid].wx, mats[fid].wy, s);
        decoder_forward(P, latents + fid * LATENT, s, ang, 0, &A);
        decoder_backward(P, &A, dy, grad_dec, dzp);
        for (int k = 0; k < LATENT; k++)
            grad_latent[fid * LATENT + k] += dzp[k];
    }
}

/* Loss of Eq. (9)-(11) of the paper-size decoder on a batch with per-fabric
 * latents z[nmats][64] (trained directly as parameters), and its gradient:
 * grad [N_PDEC] and dlatent [nmats][64].  Faulted samples contribute
 * nothing but count in n.  Returns the loss. */
double orc_paper_loss_grad(const double *P, const double *latents, const orc_material *mats,
                           int nmats, const orc_gbuffer *g, int raw, int fused,
                           const float *targets, double *grad, double *dlatent)
{
    int64_t n = g->n;
#ifdef _OPENMP
    int nth = omp_get_max_threads();
#else
    int nth = 1;
#endif
    double *Gt = (double *)calloc((size_t)nth * N_PDEC, sizeof(double));
    double *dzt = (double *)calloc((size_t)nth * nmats * PLATENT + 1, sizeof(double));
    double *lt = (double *)calloc((size_t)nth, sizeof(double));
#pragma omp parallel
    {
#ifdef _OPENMP
        int tid = omp_get_thread_num();
#else
        int tid = 0;
#endif
        double *G = Gt + (size_t)tid * N_PDEC;
        double *dzl = dzt + (size_t)tid * nmats * PLATENT;
#pragma omp for schedule(static)
        for (int64_t p = 0; p < n; p++) {
            int fid;
            double u, v, r, wi[3], wo[3];
            load_pixel(g, p, &fid, &u, &v, &r, wi, wo);
            if (pixel_fault(nmats, fid, u, v, r, wi, wo))
                continue;
            double f[PBLOB], ang[NANG] = {wi[0], wi[1], wi[2], wo[0], wo[1]};
            double tgt[4], dy[NOUT], dzp[PLATENT];
            for (int c = 0; c < 4; c++)
                tgt[c] = targets[(int64_t)c * n + p];
            paper_acts A;
            (raw ? orc_paper_features_raw : orc_paper_features)(u, v, r, mats[fid].wx, mats[fid].wy, f);
            paper_forward_acts(P, latents + (int64_t)fid * PLATENT, f, ang, fused, 0, &A);
            lt[tid] += loss_terms(A.y, tgt, spec_k(wi[2]), n, dy);
            paper_backward(P, &A, dy, G, dzp);
            for (int k = 0; k < PLATENT; k++)
                dzl[fid * PLATENT + k] += dzp[k];
        }
    }
    /* Fixed-order reduction of the per-thread partials. */
    double loss = 0.0;
    memset(grad, 0, sizeof(double) * N_PDEC);
    memset(dlatent, 0, sizeof(double) * nmats * PLATENT);
    for (int t = 0; t < nth; t++) {
        loss += lt[t];
        for (int k = 0; k < N_PDEC; k++)
            grad[k] += Gt[(size_t)t * N_PDEC + k];
        for (int k = 0; k < nmats * PLATENT; k++)
            dlatent[k] += dzt[(size_t)t * nmats * PLATENT + k];
    }
    free(Gt);
    free(dzt);
    free(lt);
    return loss;
}

/* ---- Adam (Kingma and Ba 2015, Algorithm 1) ------------------------------ */

/* One step t (1-based) on n parameters: FP64 moments m, v; the parameters are
 * float32 masters, updated in double and rounded back. */
void orc_adam_step(float *theta, const double *grad, double *m, double *v, int64_t n, int64_t t,
                   double lr, double beta1, double beta2, double eps)
{
    double c1 = 1.0 - pow(beta1, (double)t), c2 = 1.0 - pow(beta2, (double)t);
    for (int64_t k = 0; k < n; k++) {
        m[k] = beta1 * m[k] + (1.0 - beta1) * grad[k];
        v[k] = beta2 * v[k] + (1.0 - beta2) * grad[k] * grad[k];
        double mh = m[k] / c1, vh = v[k] / c2;
        theta[k] = (float)((double)theta[k] - lr * mh / (sqrt(vh) + eps));
    }
}

/* ---- Training-batch recipe ------------------------------------------------ */

/* Sample q of a training batch drawn from SplitMix64(seed), outputs 8q..8q+4:
 *   8q+0: fabric id = (z >> 32) mod n_fabrics
 *   8q+1: (u, v) = 8 * two 24-bit uniforms (cells)
 *   8q+2: radius = exp(ln r_lo + xi (ln r_hi - ln r_lo)), xi the upper 24-bit uniform
 *   8q+3: wi cosine-weighted from (xi1, xi2): (sqrt(xi1) cos 2 pi xi2,
 *         sqrt(xi1) sin 2 pi xi2, sqrt(1 - xi1))
 *   8q+4: wo likewise.
 * Values are computed in double and rounded to float32. */
void orc_batch_gen(uint64_t seed, int64_t n, int n_fabrics, double r_lo, double r_hi,
                   double btdf_frac, uint16_t *fid, float *u, float *v, float *r, float *wi_x,
                   float *wi_y, float *wi_z, float *wo_x, float *wo_y, float *wo_z)
{
    for (int64_t q = 0; q < n; q++) {
        uint64_t base = 8ull * (uint64_t)q;
        double a, b;
        fid[q] = (uint16_t)((orc_splitmix64(seed, base + 0) >> 32) % (uint64_t)n_fabrics);
        u24_pair(orc_splitmix64(seed, base + 1), &a, &b);
        u[q] = (float)(8.0 * a);
        v[q] = (float)(8.0 * b);
        u24_pair(orc_splitmix64(seed, base + 2), &a, &b);
        r[q] = (float)exp(log(r_lo) + a * (log(r_hi) - log(r_lo)));
        u24_pair(orc_splitmix64(seed, base + 3), &a, &b);
        wi_x[q] = (float)(sqrt(a) * cos(2.0 * ORC_PI * b));
        wi_y[q] = (float)(sqrt(a) * sin(2.0 * ORC_PI * b));
        wi_z[q] = (float)sqrt(1.0 - a);
        u24_pair(orc_splitmix64(seed, base + 4), &a, &b);
        wo_x[q] = (float)(sqrt(a) * cos(2.0 * ORC_PI * b));
        wo_y[q] = (float)(sqrt(a) * sin(2.0 * ORC_PI * b));
        wo_z[q] = (float)sqrt(1.0 - a);
        /* Output 8q+5 lights the sample from below with probability btdf_frac. */
        u24_pair(orc_splitmix64(seed, base + 5), &a, &b);
        if (a < btdf_frac)
            wi_z[q] = -wi_z[q];
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n);
#else
    (void)n;
#endif
}
