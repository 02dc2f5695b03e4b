/*
 * raypc_oracle.c -- plain, slow, FP64 reference ray caster.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the tests, the smoke check and the benchmark's CPU-baseline
 * leg do.  It shares no code, header or table with the HIP library.
 *
 * What it computes (paper, Section 2.2 "Rendering"): direct volume ray casting
 * of a multi-variable volume in which every sample is tested against the
 * per-variable lower/upper bounds the user set in the parallel-coordinates
 * plot; a sample that does not satisfy them is discarded and contributes
 * nothing to the ray's colour (brushing, Section 2).  Samples that pass are
 * classified through a transfer function on one chosen variable (Section 3,
 * Tasks 1-5, which colour by radial velocity, density anomaly or temperature
 * anomaly) and composited.  The geometry is the spherical shell of a planetary
 * mantle (abstract, Section 1).
 *
 * The paper gives no formulas; the discrete definition below is the reading
 * written down in the design notes (grid, shell, sample placement, trilinear
 * fetch with clamp to edge, inclusive brush, 256-entry piecewise-linear RGBA
 * table, opacity correction to a reference length, front-to-back "over"
 * compositing with early termination), evaluated step by step in double
 * precision, one pixel at a time, with no skipping, no blocking and no reuse.
 *
 * Every output is per requested pixel: premultiplied RGBA, the nominal sample
 * count (samples visited up to and including an early-termination stop), the
 * composited count (samples that passed the brush and had non-zero table
 * opacity), the marched length (sum of sample lengths), the depth that image
 * warping reprojects with (the mean distance from the eye of the composited
 * samples, each weighted by its contribution to the pixel's opacity; the paper,
 * Sections 2 and 2.2, warps the last image to fill frames the renderer has not
 * delivered yet and names no depth, so this opacity-weighted mean is the reading
 * taken here) and a fragility mask naming decisions that sit within
 * floating-point reach of a threshold:
 *   bit 0  a brush comparison within delta_b of its bound that could flip the
 *          sample's outcome (delta_b grows with the segment's grazing reach,
 *          below; for a coordinate axis delta_b = 1e-5 plus that reach, in world
 *          units),
 *   bit 1  accumulated opacity within 1e-4 of the termination threshold,
 *   bit 2  a ray grazing the inner or outer sphere (|discriminant| <= 1e-5),
 *   bit 3  a segment length within 1e-5 (world units) plus the grazing reach
 *          of its two ends of a whole number of steps (affects the sample count
 *          only),
 *   bit 4  a table lookup within 0.05 entries of a zero / non-zero opacity
 *          boundary.
 * Bits 0 and 1 are decisions with two legitimate outcomes each: oracle_outcomes
 * renders a pixel again with any of them (up to a limit) taken the other way, so
 * that a renderer's result on such a pixel can be checked against the set of
 * results the definition admits there (reading of the paper's Section 2.2: a
 * sample either passes the brush and is composited or is discarded; a float32
 * renderer may decide a sample within floating-point reach of a bound either way).
 * Grazing reach: a renderer working in float32 (unit roundoff u = 2^-24) finds
 * a sphere hit from the closest-approach discriminant r^2 - |p|^2, p = o - (o.d) d,
 * which cancels for rays that nearly graze the sphere: a few ulps of error in p
 * move the roots by about 4 u (|o| + r) r / sqrt(disc) world units.  Near-tangent
 * chords therefore have ill-conditioned ends in float32 however the renderer
 * orders its operations, and both their sample count and the positions of their
 * samples are legitimately uncertain by that much.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_FIELDS 8

typedef struct {
    int n_fields, n;
    const float *const *fields;
    double maxabs[ORACLE_MAX_FIELDS];
    double r_inner, r_outer;
    const uint8_t *active;
    const double *lo, *hi;
    const uint8_t *coord_active; /* 4 or NULL: brush on the sample position x, y, z and radius */
    const double *coord_lo, *coord_hi;
    int tf_field;
    double vmin, vmax, ref_step;
    const double *tf; /* 256 x 4 straight RGBA */
    double ert;
    const double *bg; /* 4 or NULL */
    double eye[3], fwd[3], right[3], upv[3], tan_half, aspect;
    int width, height;
    double step_vox;
} oracle_params;

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static void normalize3(double *a)
{
    double l = sqrt(dot3(a, a));
    a[0] /= l;
    a[1] /= l;
    a[2] /= l;
}

static double voxel(const float *v, int n, long z, long y, long x)
{
    return (double)v[(z * n + y) * n + x];
}

static long clampi(long i, int n)
{
    return i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
}

/* Trilinear interpolation at continuous voxel index u = (ux,uy,uz): corners
 * floor(u) and floor(u)+1, each clamped to [0, n-1]; weights from the
 * unclamped floor.  Also reports max - min over the eight corners. */
static double trilinear(const float *v, int n, double ux, double uy, double uz, double *corner_range)
{
    double fx = floor(ux), fy = floor(uy), fz = floor(uz);
    double wx = ux - fx, wy = uy - fy, wz = uz - fz;
    long x0 = clampi((long)fx, n), x1 = clampi((long)fx + 1, n);
    long y0 = clampi((long)fy, n), y1 = clampi((long)fy + 1, n);
    long z0 = clampi((long)fz, n), z1 = clampi((long)fz + 1, n);
    double c[8] = {voxel(v, n, z0, y0, x0), voxel(v, n, z0, y0, x1), voxel(v, n, z0, y1, x0),
                   voxel(v, n, z0, y1, x1), voxel(v, n, z1, y0, x0), voxel(v, n, z1, y0, x1),
                   voxel(v, n, z1, y1, x0), voxel(v, n, z1, y1, x1)};
    double r = 0.0;
    for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b)
            if (fabs(c[a] - c[b]) > r) r = fabs(c[a] - c[b]);
    if (corner_range) *corner_range = r;
    double val = 0.0;
    for (int k = 0; k < 8; ++k) {
        double w = ((k & 1) ? wx : 1.0 - wx) * ((k & 2) ? wy : 1.0 - wy) * ((k & 4) ? wz : 1.0 - wz);
        val += w * c[k];
    }
    return val;
}

/* Exported for the affine-field pin: values at npts continuous voxel indices. */
void oracle_trilinear(const float *v, int n, const double *u_xyz, int npts, double *out)
{
    for (int i = 0; i < npts; ++i)
        out[i] = trilinear(v, n, u_xyz[3 * i], u_xyz[3 * i + 1], u_xyz[3 * i + 2], NULL);
}

/* Intersection of the line o + t d (|d| = 1) with the sphere of radius rho,
 * written as the textbook quadratic t^2 + 2 b t + c = 0.  Returns the
 * discriminant; the hit interval is [t0, t1] when it is positive. */
static double sphere(const double *o, const double *d, double rho, double *t0, double *t1)
{
    double b = dot3(o, d);
    double c = dot3(o, o) - rho * rho;
    double disc = b * b - c;
    if (disc > 0.0) {
        double s = sqrt(disc);
        *t0 = -b - s;
        *t1 = -b + s;
    }
    return disc;
}

typedef struct {
    double rgba[4];
    uint32_t nominal, composited;
    uint8_t fragile;
    double pathlen;
    double depth; /* opacity-weighted mean distance of the composited samples; +inf if none */
} pixel_result;

/* Flippable decisions (fragile bits 0 and 1) met while rendering a pixel, in the order met:
 * decision i is taken the other way when i < n_forced and forced[i] is set.  NULL: every
 * decision as the double-precision arithmetic takes it. */
typedef struct {
    const uint8_t *forced;
    int n_forced;
    int seen; /* decisions met so far */
} decisions;

static int decide(decisions *dc, int outcome)
{
    if (!dc) return outcome;
    int i = dc->seen++;
    return (i < dc->n_forced && dc->forced[i]) ? !outcome : outcome;
}

/* Float32 reach of a root of the sphere of radius rho with discriminant disc (see the header). */
static double graze_reach(double o_norm, double rho, double disc)
{
    return disc > 0.0 ? 4.0 * ldexp(1.0, -24) * (o_norm + rho) * rho / sqrt(disc) : 0.0;
}

/* `jit` is the pixel's sample-grid offset s in [0, 1) (in steps): samples of a segment [a, b] are
 * the pieces of [a, b] cut at g + j ds (g = a - s ds), each evaluated at its midpoint; s = 0 gives
 * the regular partition. */
static void render_pixel(const oracle_params *P, int px, int py, double jit, pixel_result *res, decisions *dc)
{
    memset(res, 0, sizeof(*res));
    /* ray through the pixel centre; row 0 is the top row */
    double sx = (2.0 * (px + 0.5) / P->width - 1.0) * P->tan_half * P->aspect;
    double sy = (1.0 - 2.0 * (py + 0.5) / P->height) * P->tan_half;
    double d[3], o[3];
    for (int k = 0; k < 3; ++k) {
        d[k] = P->fwd[k] + sx * P->right[k] + sy * P->upv[k];
        o[k] = P->eye[k];
    }
    normalize3(d);

    /* shell = outer ball minus the open inner ball, restricted to t >= 0 */
    double seg[2][2], reach[2][2];
    int nseg = 0;
    double t0 = 0, t1 = 0, s0 = 0, s1 = 0;
    double disc_out = sphere(o, d, P->r_outer, &t0, &t1);
    double disc_in = P->r_inner > 0.0 ? sphere(o, d, P->r_inner, &s0, &s1) : -1.0;
    if (fabs(disc_out) <= 1e-5 || (P->r_inner > 0.0 && fabs(disc_in) <= 1e-5)) res->fragile |= 4;
    if (disc_out > 0.0) {
        const double o_norm = sqrt(dot3(o, o));
        const double r_out_reach = graze_reach(o_norm, P->r_outer, disc_out);
        const double r_in_reach = graze_reach(o_norm, P->r_inner, disc_in);
        double cand[2][2], cr[2][2];
        int nc = 0;
        if (disc_in > 0.0) {
            cand[nc][0] = t0;
            cand[nc][1] = fmin(t1, s0);
            cr[nc][0] = r_out_reach;
            cr[nc][1] = s0 < t1 ? r_in_reach : r_out_reach;
            ++nc;
            cand[nc][0] = fmax(t0, s1);
            cand[nc][1] = t1;
            cr[nc][0] = s1 > t0 ? r_in_reach : r_out_reach;
            cr[nc][1] = r_out_reach;
            ++nc;
        } else {
            cand[nc][0] = t0;
            cand[nc][1] = t1;
            cr[nc][0] = r_out_reach;
            cr[nc][1] = r_out_reach;
            ++nc;
        }
        for (int k = 0; k < nc; ++k) {
            double a = fmax(cand[k][0], 0.0), b = cand[k][1];
            if (b > a) {
                seg[nseg][0] = a;
                seg[nseg][1] = b;
                reach[nseg][0] = cand[k][0] < 0.0 ? 0.0 : cr[k][0];  /* a start clipped at the eye is exact */
                reach[nseg][1] = cr[k][1];
                ++nseg;
            }
        }
    }

    const int n = P->n;
    const double h = 2.0 / n;
    const double ds = P->step_vox * h;
    double C[3] = {0, 0, 0}, A = 0.0, D = 0.0;
    int done = 0;
    for (int sgi = 0; sgi < nseg && !done; ++sgi) {
        double a = seg[sgi][0], b = seg[sgi][1];
        double g = a - jit * ds;
        double q = (b - g) / ds;
        long ns = (long)ceil(q);
        if (fabs((b - g) - ds * nearbyint(q)) <= 1e-5 + reach[sgi][0] + reach[sgi][1]) res->fragile |= 8;
        /* grazing reach of the segment's ends in voxels: how far float32 may move its samples */
        const double pos_reach = fmax(reach[sgi][0], reach[sgi][1]) / h;
        for (long j = 0; j < ns && !done; ++j) {
            double tlo = fmax(a, g + j * ds);
            double thi = fmin(g + (j + 1) * ds, b);
            double len = thi - tlo;
            double tm = 0.5 * (tlo + thi);
            double u[3];
            for (int k = 0; k < 3; ++k) u[k] = (o[k] + d[k] * tm + 1.0) / h - 0.5;
            res->nominal++;
            res->pathlen += len;

            /* brush: every active variable must lie inside [lo, hi] */
            int robust_fail = 0, near = 0, pass = 1;
            double tf_value = 0.0;
            int have_tf = 0;
            for (int f = 0; f < P->n_fields; ++f) {
                if (!P->active[f]) continue;
                double rng;
                double v = trilinear(P->fields[f], n, u[0], u[1], u[2], &rng);
                if (f == P->tf_field) {
                    tf_value = v;
                    have_tf = 1;
                }
                int ok = (v >= P->lo[f]) && (v <= P->hi[f]);
                if (!ok) pass = 0;
                double dlo = (1e-3 + 2.0 * pos_reach) * rng + ldexp(fmax(fabs(P->lo[f]), P->maxabs[f]), -20);
                double dhi = (1e-3 + 2.0 * pos_reach) * rng + ldexp(fmax(fabs(P->hi[f]), P->maxabs[f]), -20);
                int near_f = (fabs(v - P->lo[f]) <= dlo) || (fabs(v - P->hi[f]) <= dhi);
                if (near_f)
                    near = 1;
                else if (!ok)
                    robust_fail = 1;
            }
            if (P->coord_active) {
                /* coordinate axes: the sample position (world x, y, z) and its radius */
                double p[3], pr = 0.0;
                for (int k = 0; k < 3; ++k) {
                    p[k] = o[k] + d[k] * tm;
                    pr += p[k] * p[k];
                }
                pr = sqrt(pr);
                const double dc = 1e-5 + pos_reach * h;
                for (int ax = 0; ax < 4; ++ax) {
                    if (!P->coord_active[ax]) continue;
                    const double v = ax < 3 ? p[ax] : pr;
                    int ok = (v >= P->coord_lo[ax]) && (v <= P->coord_hi[ax]);
                    if (!ok) pass = 0;
                    int near_c = (fabs(v - P->coord_lo[ax]) <= dc) || (fabs(v - P->coord_hi[ax]) <= dc);
                    if (near_c)
                        near = 1;
                    else if (!ok)
                        robust_fail = 1;
                }
            }
            if (near && !robust_fail) {
                res->fragile |= 1;
                pass = decide(dc, pass);
            }
            if (!pass) continue; /* discarded: counted, not composited */

            if (!have_tf) tf_value = trilinear(P->fields[P->tf_field], n, u[0], u[1], u[2], NULL);
            double x = (tf_value - P->vmin) / (P->vmax - P->vmin);
            x = x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x);
            x *= 255.0;
            int i = (int)floor(x);
            if (i > 254) i = 254;
            double w = x - i;
            double s[4];
            for (int c = 0; c < 4; ++c) s[c] = (1.0 - w) * P->tf[4 * i + c] + w * P->tf[4 * (i + 1) + c];
            {
                int klo = (int)floor(fmax(x - 0.05, 0.0)), khi = (int)ceil(x + 0.05);
                if (khi > 255) khi = 255;
                int has0 = 0, has1 = 0;
                for (int k = klo; k <= khi; ++k) {
                    if (P->tf[4 * k + 3] == 0.0)
                        has0 = 1;
                    else
                        has1 = 1;
                }
                if (has0 && has1) res->fragile |= 16;
            }
            if (s[3] > 0.0) res->composited++;
            /* opacity of the table is per reference length; correct to len */
            double alpha = s[3] >= 1.0 ? 1.0 : -expm1((len / P->ref_step) * log1p(-s[3]));
            if (alpha == 0.0) continue;
            for (int c = 0; c < 3; ++c) C[c] += (1.0 - A) * alpha * s[c];
            D += (1.0 - A) * alpha * tm;
            A += (1.0 - A) * alpha;
            if (P->ert < 1.0) {
                int stop = A >= P->ert;
                if (fabs(A - P->ert) <= 1e-4) {
                    res->fragile |= 2;
                    stop = decide(dc, stop);
                }
                if (stop) done = 1;
            }
        }
    }
    /* depth: the sample distances tm weighted by each sample's share (1 - A) alpha of the final
     * opacity, whose sum is A; taken before the background, which has no depth */
    res->depth = A > 0.0 ? D / A : INFINITY;
    if (P->bg) {
        for (int c = 0; c < 3; ++c) C[c] += (1.0 - A) * P->bg[c];
        A += (1.0 - A) * P->bg[3];
    }
    res->rgba[0] = C[0];
    res->rgba[1] = C[1];
    res->rgba[2] = C[2];
    res->rgba[3] = A;
}

/* Fill the parameters of a render; -1 on invalid arguments. */
static int setup(oracle_params *P, int n_fields, int n, const float *const *fields, double r_inner, double r_outer,
                 const uint8_t *active, const double *lo, const double *hi, const uint8_t *coord_active,
                 const double *coord_lo, const double *coord_hi, int tf_field, double vmin, double vmax,
                 const double *tf_rgba, double ref_step, double ert, const double *bg, const double *camera,
                 int width, int height, double step_vox)
{
    if (n_fields < 1 || n_fields > ORACLE_MAX_FIELDS || n < 2 || width < 1 || height < 1 ||
        tf_field < 0 || tf_field >= n_fields || !(vmax > vmin) || !(step_vox > 0) || !(ref_step > 0))
        return -1;
    memset(P, 0, sizeof(*P));
    P->n_fields = n_fields;
    P->n = n;
    P->fields = fields;
    for (int f = 0; f < n_fields; ++f) {
        double m = 0.0;
        size_t cnt = (size_t)n * n * n;
        for (size_t i = 0; i < cnt; ++i)
            if (fabs((double)fields[f][i]) > m) m = fabs((double)fields[f][i]);
        P->maxabs[f] = m;
    }
    P->r_inner = r_inner;
    P->r_outer = r_outer;
    P->active = active;
    P->lo = lo;
    P->hi = hi;
    P->coord_active = coord_active;
    P->coord_lo = coord_lo;
    P->coord_hi = coord_hi;
    P->tf_field = tf_field;
    P->vmin = vmin;
    P->vmax = vmax;
    P->tf = tf_rgba;
    P->ref_step = ref_step;
    P->ert = ert;
    P->bg = bg;
    P->width = width;
    P->height = height;
    P->step_vox = step_vox;
    double up[3];
    for (int k = 0; k < 3; ++k) {
        P->eye[k] = camera[k];
        P->fwd[k] = camera[3 + k] - camera[k];
        up[k] = camera[6 + k];
    }
    normalize3(P->fwd);
    cross3(P->fwd, up, P->right);
    normalize3(P->right);
    cross3(P->right, P->fwd, P->upv);
    P->tan_half = tan(0.5 * camera[9] * M_PI / 180.0);
    P->aspect = (double)width / (double)height;

    return 0;
}

/*
 * oracle_render: render the listed pixels (linear index py*width + px; NULL
 * means every pixel in row-major order).  `fields` are the level's stored
 * values already converted to float32 ([z][y][x], n^3 each).  Camera is
 * {eye[3], target[3], up[3], fov_y_deg}.  `coord_active` (4 flags or NULL) with
 * `coord_lo` / `coord_hi` restricts the sample position: axes 0..2 its world x, y,
 * z, axis 3 its radius.  `bg` may be NULL.  `jitter` holds
 * one sample-grid offset in [0, 1) per requested pixel (NULL: 0, the regular
 * partition).  `depth` receives the opacity-weighted mean sample distance from
 * the eye (+inf where nothing was composited).  Any output pointer may be NULL.
 * Returns 0, or -1 on invalid arguments.
 */
int oracle_render(int n_fields, int n, const float *const *fields, double r_inner, double r_outer,
                  const uint8_t *active, const double *lo, const double *hi, const uint8_t *coord_active,
                  const double *coord_lo, const double *coord_hi, int tf_field, double vmin,
                  double vmax, const double *tf_rgba, double ref_step, double ert, const double *bg,
                  const double *camera, int width, int height, double step_vox, long n_pix,
                  const int64_t *pix, const double *jitter, double *rgba, uint32_t *nominal,
                  uint32_t *composited, uint8_t *fragile, double *pathlen, double *depth, int n_threads)
{
    oracle_params P;
    if (setup(&P, n_fields, n, fields, r_inner, r_outer, active, lo, hi, coord_active, coord_lo, coord_hi, tf_field,
              vmin, vmax, tf_rgba, ref_step, ert, bg, camera, width, height, step_vox) != 0)
        return -1;

    long total = pix ? n_pix : (long)width * height;
#pragma omp parallel for schedule(dynamic, 64) num_threads(n_threads > 0 ? n_threads : 1)
    for (long k = 0; k < total; ++k) {
        long lin = pix ? (long)pix[k] : k;
        pixel_result r;
        render_pixel(&P, (int)(lin % width), (int)(lin / width), jitter ? jitter[k] : 0.0, &r, NULL);
        if (rgba)
            for (int c = 0; c < 4; ++c) rgba[4 * k + c] = r.rgba[c];
        if (nominal) nominal[k] = r.nominal;
        if (composited) composited[k] = r.composited;
        if (fragile) fragile[k] = r.fragile;
        if (pathlen) pathlen[k] = r.pathlen;
        if (depth) depth[k] = r.depth;
    }
    return 0;
}

/*
 * Outcomes of near-threshold decisions.  A pixel's flippable decisions (fragile
 * bits 0 and 1) each admit two results; the pixel's legitimate results are the
 * renders with any set of them taken the other way.  They are enumerated depth
 * first: a render that follows `choice` for its first `len` decisions (the rest
 * as double precision takes them) is one outcome, and its children take one more
 * decision i >= len the other way, the decisions between len and i as double
 * precision takes them; every set of flipped decisions is met exactly once.  At
 * most `max_flips` decisions are flipped on one path, and at most `max_out`
 * outcomes are kept.
 */
#define ORACLE_MAX_DECISIONS 8192

typedef struct {
    const oracle_params *P;
    int px, py;
    double jit;
    int max_flips, max_out;
    uint8_t *choice;
    pixel_result *outs;
    uint8_t *flips;
    int n_out;
} explore_state;

static int explore(explore_state *E, int len, int flips)
{
    if (E->n_out >= E->max_out) return -1;
    decisions dc = {E->choice, len, 0};
    render_pixel(E->P, E->px, E->py, E->jit, &E->outs[E->n_out], &dc);
    E->flips[E->n_out] = (uint8_t)flips;
    E->n_out++;
    if (flips >= E->max_flips) return 0;
    for (int i = len; i < dc.seen; ++i) {
        if (i >= ORACLE_MAX_DECISIONS) return -1;
        memset(E->choice + len, 0, (size_t)(i - len));
        E->choice[i] = 1;
        if (explore(E, i + 1, flips + 1) != 0) return -1;
    }
    return 0;
}

/*
 * oracle_outcomes: for each listed pixel (linear index py*width + px, with its
 * jitter offset or NULL), every outcome with at most `max_flips` of its
 * flippable decisions taken the other way: n_outcomes[k] outcomes (the first is
 * the double-precision result itself), or -1 when there are more than `max_out`
 * or a path meets more than 8192 decisions.  Outcome o of pixel k is at
 * rgba[(k max_out + o) 4 ...], nominal / composited / depth / flips[k max_out + o]
 * (flips: how many decisions that outcome takes the other way).  Other
 * arguments as oracle_render.  Returns 0, or -1 on invalid arguments.
 */
int oracle_outcomes(int n_fields, int n, const float *const *fields, double r_inner, double r_outer,
                    const uint8_t *active, const double *lo, const double *hi, const uint8_t *coord_active,
                    const double *coord_lo, const double *coord_hi, int tf_field, double vmin, double vmax,
                    const double *tf_rgba, double ref_step, double ert, const double *bg, const double *camera,
                    int width, int height, double step_vox, long n_pix, const int64_t *pix, const double *jitter,
                    int max_flips, int max_out, int32_t *n_outcomes, double *rgba, uint32_t *nominal,
                    uint32_t *composited, double *depth, uint8_t *flips, int n_threads)
{
    oracle_params P;
    if (!pix || max_out < 1 || max_flips < 0 ||
        setup(&P, n_fields, n, fields, r_inner, r_outer, active, lo, hi, coord_active, coord_lo, coord_hi, tf_field,
              vmin, vmax, tf_rgba, ref_step, ert, bg, camera, width, height, step_vox) != 0)
        return -1;
#pragma omp parallel num_threads(n_threads > 0 ? n_threads : 1)
    {
        uint8_t *choice = (uint8_t *)calloc(ORACLE_MAX_DECISIONS, 1);
        pixel_result *outs = (pixel_result *)malloc(sizeof(pixel_result) * (size_t)max_out);
        uint8_t *fl = (uint8_t *)malloc((size_t)max_out);
#pragma omp for schedule(dynamic, 1)
        for (long k = 0; k < n_pix; ++k) {
            long lin = (long)pix[k];
            explore_state E = {&P, (int)(lin % width), (int)(lin / width), jitter ? jitter[k] : 0.0,
                               max_flips, max_out, choice, outs, fl, 0};
            int ok = choice && outs && fl && explore(&E, 0, 0) == 0;
            n_outcomes[k] = ok ? E.n_out : -1;
            for (int o = 0; ok && o < E.n_out; ++o) {
                size_t at = (size_t)k * max_out + o;
                for (int c = 0; c < 4; ++c) rgba[4 * at + c] = outs[o].rgba[c];
                nominal[at] = outs[o].nominal;
                composited[at] = outs[o].composited;
                depth[at] = outs[o].depth;
                flips[at] = fl[o];
            }
        }
        free(choice);
        free(outs);
        free(fl);
    }
    return 0;
}
