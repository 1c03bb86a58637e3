/*
 * Synthetic-input generator: exact line integrals and voxel averages of a
 * phantom made of rotated ellipsoids and axis-aligned boxes.
 *
 * This file produces *inputs* only (measured data and ground truth for the
 * synthetic workloads).  It contains nothing of the reconstruction method.
 *
 * Ellipsoid record (16 doubles): centre c[3], rotation R[9] (row-major; the
 * columns are the body axes in world coordinates), semi-axes a[3], kappa.
 * Box record (7 doubles): lo[3], hi[3], kappa.
 * View record (12 doubles): source s[3], detector centre d[3], column step
 * u[3], row step v[3].  Pixel (a,b) is centred at
 * d + (a-(nu-1)/2) u + (b-(nv-1)/2) v, and the ray runs from s to it.
 */
#include <math.h>
#include <stddef.h>

#define ELL_STRIDE 16
#define BOX_STRIDE 7

/* Length of the part of segment s -> s+D (t in [0,1]) inside the ellipsoid. */
static double ellipsoid_chord(const double *e, const double s[3], const double D[3])
{
    const double *c = e, *R = e + 3, *ax = e + 12;
    double sp[3], dp[3];
    for (int k = 0; k < 3; ++k) {
        /* body coordinates: R^T (x - c), scaled by 1/a */
        double ps = 0.0, pd = 0.0;
        for (int r = 0; r < 3; ++r) {
            ps += R[r * 3 + k] * (s[r] - c[r]);
            pd += R[r * 3 + k] * D[r];
        }
        sp[k] = ps / ax[k];
        dp[k] = pd / ax[k];
    }
    double A = dp[0] * dp[0] + dp[1] * dp[1] + dp[2] * dp[2];
    double B = 2.0 * (sp[0] * dp[0] + sp[1] * dp[1] + sp[2] * dp[2]);
    double C = sp[0] * sp[0] + sp[1] * sp[1] + sp[2] * sp[2] - 1.0;
    double disc = B * B - 4.0 * A * C;
    if (disc <= 0.0 || A <= 0.0) return 0.0;
    double r = sqrt(disc);
    double t0 = (-B - r) / (2.0 * A), t1 = (-B + r) / (2.0 * A);
    if (t0 < 0.0) t0 = 0.0;
    if (t1 > 1.0) t1 = 1.0;
    if (t1 <= t0) return 0.0;
    return (t1 - t0) * sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
}

/* Slab method for an axis-aligned box. */
static double box_chord(const double *b, const double s[3], const double D[3])
{
    double t0 = 0.0, t1 = 1.0;
    for (int k = 0; k < 3; ++k) {
        if (D[k] == 0.0) {
            if (s[k] < b[k] || s[k] > b[3 + k]) return 0.0;
            continue;
        }
        double ta = (b[k] - s[k]) / D[k], tb = (b[3 + k] - s[k]) / D[k];
        if (ta > tb) { double t = ta; ta = tb; tb = t; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
    }
    if (t1 <= t0) return 0.0;
    return (t1 - t0) * sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
}

/* Parameter interval [t0, t1] of the segment inside an axis-aligned box. */
static void box_interval(const double *lo, const double *hi, const double s[3], const double D[3],
                         double *t0, double *t1)
{
    double a = 0.0, b = 1.0;
    for (int k = 0; k < 3; ++k) {
        if (D[k] == 0.0) {
            if (s[k] < lo[k] || s[k] > hi[k]) { a = 1.0; b = 0.0; }
            continue;
        }
        double ta = (lo[k] - s[k]) / D[k], tb = (hi[k] - s[k]) / D[k];
        if (ta > tb) { double t = ta; ta = tb; tb = t; }
        if (ta > a) a = ta;
        if (tb < b) b = tb;
    }
    *t0 = a;
    *t1 = b;
}

/* Like ellipsoid_chord, restricted to t in [c0, c1]. */
static double ellipsoid_chord_clipped(const double *e, const double s[3], const double D[3], double c0, double c1)
{
    const double *c = e, *R = e + 3, *ax = e + 12;
    double sp[3], dp[3];
    for (int k = 0; k < 3; ++k) {
        double ps = 0.0, pd = 0.0;
        for (int r = 0; r < 3; ++r) {
            ps += R[r * 3 + k] * (s[r] - c[r]);
            pd += R[r * 3 + k] * D[r];
        }
        sp[k] = ps / ax[k];
        dp[k] = pd / ax[k];
    }
    double A = dp[0] * dp[0] + dp[1] * dp[1] + dp[2] * dp[2];
    double B = 2.0 * (sp[0] * dp[0] + sp[1] * dp[1] + sp[2] * dp[2]);
    double C = sp[0] * sp[0] + sp[1] * sp[1] + sp[2] * sp[2] - 1.0;
    double disc = B * B - 4.0 * A * C;
    if (disc <= 0.0 || A <= 0.0) return 0.0;
    double r = sqrt(disc);
    double t0 = (-B - r) / (2.0 * A), t1 = (-B + r) / (2.0 * A);
    if (t0 < c0) t0 = c0;
    if (t1 > c1) t1 = c1;
    if (t1 <= t0) return 0.0;
    return (t1 - t0) * sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
}

/*
 * Line integrals of the phantom restricted to the box [clip[0..2], clip[3..5]]
 * (every shape intersected with the box).
 */
void synth_line_integrals_clipped(int n_views, const double *views, int nu, int nv,
                                  int n_ell, const double *ell, int n_box, const double *box,
                                  const double *clip, double *out)
{
    long total = (long)n_views * nv * nu;
#pragma omp parallel for schedule(static)
    for (long r = 0; r < total; ++r) {
        int a = (int)(r % nu);
        int b = (int)((r / nu) % nv);
        int v = (int)(r / ((long)nu * nv));
        const double *g = views + (size_t)v * 12;
        double ca = a - 0.5 * (nu - 1), cb = b - 0.5 * (nv - 1);
        double D[3];
        for (int k = 0; k < 3; ++k) D[k] = g[3 + k] + ca * g[6 + k] + cb * g[9 + k] - g[k];
        double c0, c1;
        box_interval(clip, clip + 3, g, D, &c0, &c1);
        double acc = 0.0;
        if (c1 > c0) {
            for (int e = 0; e < n_ell; ++e) {
                const double *E = ell + (size_t)e * ELL_STRIDE;
                double ch = ellipsoid_chord_clipped(E, g, D, c0, c1);
                if (ch > 0.0) acc += E[15] * ch;
            }
            for (int e = 0; e < n_box; ++e) {
                const double *Bx = box + (size_t)e * BOX_STRIDE;
                double lo[3], hi[3];
                for (int k = 0; k < 3; ++k) {
                    lo[k] = Bx[k] > clip[k] ? Bx[k] : clip[k];
                    hi[k] = Bx[3 + k] < clip[3 + k] ? Bx[3 + k] : clip[3 + k];
                }
                if (lo[0] >= hi[0] || lo[1] >= hi[1] || lo[2] >= hi[2]) continue;
                double t0, t1;
                box_interval(lo, hi, g, D, &t0, &t1);
                if (t1 > t0) acc += Bx[6] * (t1 - t0) * sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
            }
        }
        out[r] = acc;
    }
}

/* out[v][b][a] = sum_k kappa_k * chord_k(ray(v,a,b)). */
void synth_line_integrals(int n_views, const double *views, int nu, int nv,
                          int n_ell, const double *ell, int n_box, const double *box,
                          double *out)
{
    long total = (long)n_views * nv * nu;
#pragma omp parallel for schedule(static)
    for (long r = 0; r < total; ++r) {
        int a = (int)(r % nu);
        int b = (int)((r / nu) % nv);
        int v = (int)(r / ((long)nu * nv));
        const double *g = views + (size_t)v * 12;
        double ca = a - 0.5 * (nu - 1), cb = b - 0.5 * (nv - 1);
        double D[3];
        for (int k = 0; k < 3; ++k) D[k] = g[3 + k] + ca * g[6 + k] + cb * g[9 + k] - g[k];
        double acc = 0.0;
        for (int e = 0; e < n_ell; ++e) {
            const double *E = ell + (size_t)e * ELL_STRIDE;
            double ch = ellipsoid_chord(E, g, D);
            if (ch > 0.0) acc += E[15] * ch;
        }
        for (int e = 0; e < n_box; ++e) {
            const double *Bx = box + (size_t)e * BOX_STRIDE;
            double ch = box_chord(Bx, g, D);
            if (ch > 0.0) acc += Bx[6] * ch;
        }
        out[r] = acc;
    }
}

static int inside_ellipsoid(const double *e, const double p[3])
{
    const double *c = e, *R = e + 3, *ax = e + 12;
    double q = 0.0;
    for (int k = 0; k < 3; ++k) {
        double t = 0.0;
        for (int r = 0; r < 3; ++r) t += R[r * 3 + k] * (p[r] - c[r]);
        t /= ax[k];
        q += t * t;
    }
    return q <= 1.0;
}

/*
 * vol[z][y][x] += kappa * (fraction of ss^3 sub-samples of the voxel inside
 * the shape), for every shape.  Each ellipsoid only visits its bounding box.
 */
void synth_voxelize(int nx, int ny, int nz, double h, const double *origin,
                    int n_ell, const double *ell, int n_box, const double *box,
                    int ss, double *vol)
{
    int n[3] = {nx, ny, nz};
    double c[3];
    for (int k = 0; k < 3; ++k) c[k] = origin[k] - 0.5 * (n[k] - 1) * h;  /* centre of voxel 0 */
    double inv = 1.0 / ((double)ss * ss * ss);
    for (int e = 0; e < n_ell + n_box; ++e) {
        int is_ell = e < n_ell;
        const double *E = is_ell ? ell + (size_t)e * ELL_STRIDE : box + (size_t)(e - n_ell) * BOX_STRIDE;
        double lo[3], hi[3];
        if (is_ell) {
            double r = fmax(E[12], fmax(E[13], E[14]));
            for (int k = 0; k < 3; ++k) { lo[k] = E[k] - r; hi[k] = E[k] + r; }
        } else {
            for (int k = 0; k < 3; ++k) { lo[k] = E[k]; hi[k] = E[3 + k]; }
        }
        int i0[3], i1[3];
        for (int k = 0; k < 3; ++k) {
            i0[k] = (int)floor((lo[k] - c[k]) / h - 0.5) - 1;
            i1[k] = (int)ceil((hi[k] - c[k]) / h + 0.5) + 1;
            if (i0[k] < 0) i0[k] = 0;
            if (i1[k] > n[k] - 1) i1[k] = n[k] - 1;
        }
        double kappa = is_ell ? E[15] : E[6];
#pragma omp parallel for schedule(static)
        for (int kz = i0[2]; kz <= i1[2]; ++kz) {
            for (int ky = i0[1]; ky <= i1[1]; ++ky) {
                for (int kx = i0[0]; kx <= i1[0]; ++kx) {
                    int cnt = 0;
                    for (int sz = 0; sz < ss; ++sz)
                        for (int sy = 0; sy < ss; ++sy)
                            for (int sx = 0; sx < ss; ++sx) {
                                double p[3] = {
                                    c[0] + (kx - 0.5 + (sx + 0.5) / ss) * h,
                                    c[1] + (ky - 0.5 + (sy + 0.5) / ss) * h,
                                    c[2] + (kz - 0.5 + (sz + 0.5) / ss) * h};
                                int in;
                                if (is_ell) in = inside_ellipsoid(E, p);
                                else in = p[0] >= E[0] && p[0] <= E[3] && p[1] >= E[1] && p[1] <= E[4] &&
                                          p[2] >= E[2] && p[2] <= E[5];
                                cnt += in;
                            }
                    if (cnt) vol[((size_t)kz * ny + ky) * nx + kx] += kappa * cnt * inv;
                }
            }
        }
    }
}
