/*
 * FP64 reference (oracle) for the cone-beam projector and its adjoint.
 * TEST INFRASTRUCTURE ONLY: used by the test-suite, the smoke check and the
 * CPU baseline leg of the benchmark; never by the product library.
 *
 * Model (paper Sec. 2, eq. 1): the data of a ray is the line integral of the
 * attenuation mu along the segment from the source s to a detector-pixel
 * centre q.  The paper does not state the discretisation; this oracle uses
 * Joseph's method: with D = q - s and m the axis of largest |D_m| (ties go to
 * x, then y, then z), the ray is sampled on every voxel-centre plane of axis m
 * that lies on the segment (0 <= t <= 1), the volume is interpolated
 * bilinearly in the two other axes (zero outside the grid), and the sum of the
 * samples is multiplied by the sample spacing h |D| / |D_m|.
 * The back-projection B (paper Sec. 2.1, "adjoint to the projection
 * operator") is the exact transpose, computed here by scattering the same
 * weights ray by ray.
 *
 * Geometry: volume [nz][ny][nx] (x fastest), voxel size h, box centre o;
 * voxel (i,j,k) is centred at o + ((i,j,k) - (n-1)/2) h.  View record (12
 * doubles): s[3], d[3], u[3], v[3]; pixel (a,b) is centred at
 * d + (a-(nu-1)/2) u + (b-(nv-1)/2) v.  Stacks are [view][nv][nu].
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int n[3];
    double h;
    double o[3];
} vgeom;

static void make_vgeom(vgeom *g, int nx, int ny, int nz, double h, const double *o)
{
    g->n[0] = nx; g->n[1] = ny; g->n[2] = nz;
    g->h = h;
    for (int k = 0; k < 3; ++k) g->o[k] = o[k];
}

/* Pixel centre q and direction D = q - s of ray (a,b) of a view. */
static void ray_of(const double *view, int nu, int nv, int a, int b, double q[3], double D[3])
{
    double ca = a - 0.5 * (nu - 1), cb = b - 0.5 * (nv - 1);
    for (int k = 0; k < 3; ++k) {
        q[k] = view[3 + k] + ca * view[6 + k] + cb * view[9 + k];
        D[k] = q[k] - view[k];
    }
}

/* Axis of largest |D| component; ties go to x, then y, then z. */
int oracle_major_axis(const double D[3])
{
    double ax = fabs(D[0]), ay = fabs(D[1]), az = fabs(D[2]);
    if (ax >= ay && ax >= az) return 0;
    if (ay >= az) return 1;
    return 2;
}

static double voxel_centre(const vgeom *g, int axis, int l)
{
    return g->o[axis] + (l - 0.5 * (g->n[axis] - 1)) * g->h;
}

/*
 * Visit every (voxel, weight) pair of a ray.  mode 0: return sum w*vol;
 * mode 1: out[voxel] += w * y.  The weight includes the spacing factor.
 */
static double joseph_ray(const vgeom *g, const double s[3], const double D[3],
                         const double *vol, double *out, double y, int mode)
{
    int m = oracle_major_axis(D);
    int a = (m == 0) ? 1 : 0;          /* first in-plane axis  */
    int b = (m == 2) ? 1 : 2;          /* second in-plane axis */
    double len = sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
    double scale = g->h * len / fabs(D[m]);
    double acc = 0.0;
    for (int l = 0; l < g->n[m]; ++l) {
        double X = voxel_centre(g, m, l);
        double t = (X - s[m]) / D[m];
        if (t < 0.0 || t > 1.0) continue;
        double pa = s[a] + t * D[a];
        double pb = s[b] + t * D[b];
        /* fractional voxel indices of the sample in the two in-plane axes */
        double fa = (pa - g->o[a]) / g->h + 0.5 * (g->n[a] - 1);
        double fb = (pb - g->o[b]) / g->h + 0.5 * (g->n[b] - 1);
        if (!(fa > -1.0 && fa < g->n[a] && fb > -1.0 && fb < g->n[b])) continue;
        int ja = (int)floor(fa), jb = (int)floor(fb);
        for (int ia = ja; ia <= ja + 1; ++ia) {
            if (ia < 0 || ia >= g->n[a]) continue;
            double wa = 1.0 - fabs(fa - ia);
            for (int ib = jb; ib <= jb + 1; ++ib) {
                if (ib < 0 || ib >= g->n[b]) continue;
                double wb = 1.0 - fabs(fb - ib);
                int idx[3];
                idx[m] = l; idx[a] = ia; idx[b] = ib;
                size_t off = ((size_t)idx[2] * g->n[1] + idx[1]) * g->n[0] + idx[0];
                if (mode == 0) acc += wa * wb * vol[off];
                else out[off] += wa * wb * scale * y;
            }
        }
    }
    return acc * scale;
}

/* proj[v][b][a] = (A vol) for every ray.  Parallel over rays. */
void oracle_project(int nx, int ny, int nz, double h, const double *origin,
                    int nu, int nv, int n_views, const double *views,
                    const double *vol, double *proj)
{
    vgeom g;
    make_vgeom(&g, nx, ny, nz, h, origin);
    long total = (long)n_views * nv * nu;
#pragma omp parallel for schedule(dynamic, 256)
    for (long r = 0; r < total; ++r) {
        int a = (int)(r % nu), b = (int)((r / nu) % nv), v = (int)(r / ((long)nu * nv));
        const double *view = views + (size_t)v * 12;
        double q[3], D[3];
        ray_of(view, nu, nv, a, b, q, D);
        proj[r] = joseph_ray(&g, view, D, vol, NULL, 0.0, 0);
    }
}

/* Project a list of rays given as (view, a, b) triples. */
void oracle_project_rays(int nx, int ny, int nz, double h, const double *origin,
                         int nu, int nv, const double *views, const double *vol,
                         long n_rays, const int *rays, double *out)
{
    vgeom g;
    make_vgeom(&g, nx, ny, nz, h, origin);
#pragma omp parallel for schedule(dynamic, 16)
    for (long r = 0; r < n_rays; ++r) {
        const double *view = views + (size_t)rays[3 * r] * 12;
        double q[3], D[3];
        ray_of(view, nu, nv, rays[3 * r + 1], rays[3 * r + 2], q, D);
        out[r] = joseph_ray(&g, view, D, vol, NULL, 0.0, 0);
    }
}

/*
 * vol = A^T proj by scattering every ray's weights (exact transpose of
 * oracle_project).  Views are split over threads, each with a private
 * accumulator; the partial volumes are then summed in thread order.
 */
void oracle_backproject(int nx, int ny, int nz, double h, const double *origin,
                        int nu, int nv, int n_views, const double *views,
                        const double *proj, double *vol)
{
    vgeom g;
    make_vgeom(&g, nx, ny, nz, h, origin);
    size_t nvox = (size_t)nx * ny * nz;
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
    if (nthreads > n_views) nthreads = n_views > 0 ? n_views : 1;
#endif
    double *part = (double *)calloc(nvox * (size_t)nthreads, sizeof(double));
#pragma omp parallel num_threads(nthreads)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *mine = part + nvox * (size_t)tid;
#pragma omp for schedule(static)
        for (int v = 0; v < n_views; ++v) {
            const double *view = views + (size_t)v * 12;
            for (int b = 0; b < nv; ++b)
                for (int a = 0; a < nu; ++a) {
                    double q[3], D[3];
                    ray_of(view, nu, nv, a, b, q, D);
                    double y = proj[((size_t)v * nv + b) * nu + a];
                    if (y != 0.0) joseph_ray(&g, view, D, NULL, mine, y, 1);
                }
        }
    }
    memset(vol, 0, nvox * sizeof(double));
    for (int t = 0; t < nthreads; ++t)
        for (size_t i = 0; i < nvox; ++i) vol[i] += part[nvox * (size_t)t + i];
    free(part);
}

/*
 * Weight of voxel (i,j,k) in ray (view, a, b), straight from the definition
 * and without any index arithmetic: take the voxel's own centre plane along
 * the ray's major axis, find where the ray crosses it, and multiply the
 * spacing factor by the two hat functions of the in-plane offsets.
 */
double oracle_weight(int nx, int ny, int nz, double h, const double *origin,
                     int nu, int nv, const double *view, int a, int b, int i, int j, int k)
{
    vgeom g;
    make_vgeom(&g, nx, ny, nz, h, origin);
    double q[3], D[3];
    ray_of(view, nu, nv, a, b, q, D);
    int m = oracle_major_axis(D);
    int idx[3] = {i, j, k};
    double c[3];
    for (int t = 0; t < 3; ++t) c[t] = voxel_centre(&g, t, idx[t]);
    double t = (c[m] - view[m]) / D[m];
    if (t < 0.0 || t > 1.0) return 0.0;
    double w = h * sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]) / fabs(D[m]);
    for (int ax = 0; ax < 3; ++ax) {
        if (ax == m) continue;
        double p = view[ax] + t * D[ax];
        double hat = 1.0 - fabs(p - c[ax]) / h;
        if (hat <= 0.0) return 0.0;
        w *= hat;
    }
    return w;
}

/* Dense system matrix W[ray][voxel] for tiny problems (brute force). */
void oracle_dense_matrix(int nx, int ny, int nz, double h, const double *origin,
                         int nu, int nv, int n_views, const double *views, double *W)
{
    long nvox = (long)nx * ny * nz;
    long nray = (long)n_views * nv * nu;
#pragma omp parallel for schedule(dynamic, 4)
    for (long r = 0; r < nray; ++r) {
        int a = (int)(r % nu), b = (int)((r / nu) % nv), v = (int)(r / ((long)nu * nv));
        for (long x = 0; x < nvox; ++x) {
            int i = (int)(x % nx), j = (int)((x / nx) % ny), k = (int)(x / ((long)nx * ny));
            W[r * nvox + x] = oracle_weight(nx, ny, nz, h, origin, nu, nv, views + (size_t)v * 12, a, b, i, j, k);
        }
    }
}

/* Central projection of point P onto the detector plane of a view, in
 * fractional pixel indices.  Returns 0 if P is not in front of the source. */
static int project_point(const double *view, int nu, int nv, const double P[3], double *pa, double *pb)
{
    const double *s = view, *d = view + 3, *u = view + 6, *v = view + 9;
    double n[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
    double num = 0.0, den = 0.0;
    for (int k = 0; k < 3; ++k) {
        num += n[k] * (d[k] - s[k]);
        den += n[k] * (P[k] - s[k]);
    }
    if (den == 0.0 || num / den <= 0.0) return 0;
    double t = num / den, X[3];
    for (int k = 0; k < 3; ++k) X[k] = s[k] + t * (P[k] - s[k]) - d[k];
    double uu = 0, uv = 0, vv = 0, xu = 0, xv = 0;
    for (int k = 0; k < 3; ++k) {
        uu += u[k] * u[k]; uv += u[k] * v[k]; vv += v[k] * v[k];
        xu += X[k] * u[k]; xv += X[k] * v[k];
    }
    double det = uu * vv - uv * uv;
    *pa = (xu * vv - xv * uv) / det + 0.5 * (nu - 1);
    *pb = (xv * uu - xu * uv) / det + 0.5 * (nv - 1);
    return 1;
}

/*
 * (A^T y) at single voxels, one by one: for each view, every pixel whose
 * footprint could touch the voxel lies inside the projection of the cube of
 * half-width h around the voxel centre; the weights of those pixels are
 * taken from oracle_weight.  out[n] for voxels vox[3n..3n+2] = (i,j,k).
 */
void oracle_backproject_voxels(int nx, int ny, int nz, double h, const double *origin,
                               int nu, int nv, int n_views, const double *views,
                               const double *proj, long n_vox, const int *vox, double *out)
{
    vgeom g;
    make_vgeom(&g, nx, ny, nz, h, origin);
#pragma omp parallel for schedule(dynamic, 1)
    for (long n = 0; n < n_vox; ++n) {
        int i = vox[3 * n], j = vox[3 * n + 1], k = vox[3 * n + 2];
        double c[3] = {voxel_centre(&g, 0, i), voxel_centre(&g, 1, j), voxel_centre(&g, 2, k)};
        double acc = 0.0;
        for (int v = 0; v < n_views; ++v) {
            const double *view = views + (size_t)v * 12;
            double amin = 1e300, amax = -1e300, bmin = 1e300, bmax = -1e300;
            int ok = 1;
            for (int corner = 0; corner < 8 && ok; ++corner) {
                double P[3] = {c[0] + ((corner & 1) ? h : -h), c[1] + ((corner & 2) ? h : -h),
                               c[2] + ((corner & 4) ? h : -h)};
                double pa, pb;
                if (!project_point(view, nu, nv, P, &pa, &pb)) ok = 0;
                else {
                    if (pa < amin) amin = pa;
                    if (pa > amax) amax = pa;
                    if (pb < bmin) bmin = pb;
                    if (pb > bmax) bmax = pb;
                }
            }
            int a0 = 0, a1 = nu - 1, b0 = 0, b1 = nv - 1;
            if (ok) {
                a0 = (int)floor(amin) - 1; a1 = (int)ceil(amax) + 1;
                b0 = (int)floor(bmin) - 1; b1 = (int)ceil(bmax) + 1;
                if (a0 < 0) a0 = 0;
                if (b0 < 0) b0 = 0;
                if (a1 > nu - 1) a1 = nu - 1;
                if (b1 > nv - 1) b1 = nv - 1;
            }
            for (int b = b0; b <= b1; ++b)
                for (int a = a0; a <= a1; ++a) {
                    double w = oracle_weight(nx, ny, nz, h, origin, nu, nv, view, a, b, i, j, k);
                    if (w != 0.0) acc += w * proj[((size_t)v * nv + b) * nu + a];
                }
        }
        out[n] = acc;
    }
}

/*
 * Gradient of sum_rays g[ray] * (A vol)[ray] with respect to each view's 12
 * geometry values (s, d, u, v), from the derivative of the Joseph sum above
 * (the major axis and the set of planes are held fixed: the sum is
 * piecewise smooth).  For a sample on plane X of axis m, with D = q - s,
 * t = (X - s_m)/D_m and p = s + t D:
 *   dp_k/ds_k = 1 - t, dp_k/dq_k = t             (k in-plane)
 *   dp_k/ds_m = D_k (t - 1)/D_m, dp_k/dq_m = -D_k t / D_m
 * and the bilinear sample f has df/dp_k = (difference of the two taps along
 * k, interpolated along the other in-plane axis) / h.  The ray is
 * L * sum f with L = h |D| / |D_m|.  Pixel centre q = d + ca u + cb v, so
 * dq/dd = I, dq/du = ca I, dq/dv = cb I.  dviews[v*12 + ...] is overwritten.
 */
void oracle_project_geom_grad(int nx, int ny, int nz, double h, const double *origin,
                              int nu, int nv, int n_views, const double *views,
                              const double *vol, const double *g, double *dviews)
{
    vgeom G;
    make_vgeom(&G, nx, ny, nz, h, origin);
#pragma omp parallel for schedule(dynamic, 1)
    for (int v = 0; v < n_views; ++v) {
        const double *view = views + (size_t)v * 12;
        const double *s = view;
        double acc[12] = {0};
        for (int b = 0; b < nv; ++b)
            for (int a = 0; a < nu; ++a) {
                double gr = g[((size_t)v * nv + b) * nu + a];
                if (gr == 0.0) continue;
                double q[3], D[3];
                ray_of(view, nu, nv, a, b, q, D);
                int m = oracle_major_axis(D);
                int ax[2] = {(m == 0) ? 1 : 0, (m == 2) ? 1 : 2};
                double len = sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
                double L = h * len / fabs(D[m]);
                double sum = 0.0, ds[3] = {0, 0, 0}, dq[3] = {0, 0, 0};
                for (int l = 0; l < G.n[m]; ++l) {
                    double X = voxel_centre(&G, m, l);
                    double t = (X - s[m]) / D[m];
                    if (t < 0.0 || t > 1.0) continue;
                    double f[2];
                    int j[2];
                    for (int c = 0; c < 2; ++c) {
                        double p = s[ax[c]] + t * D[ax[c]];
                        f[c] = (p - G.o[ax[c]]) / h + 0.5 * (G.n[ax[c]] - 1);
                    }
                    if (!(f[0] > -1.0 && f[0] < G.n[ax[0]] && f[1] > -1.0 && f[1] < G.n[ax[1]])) continue;
                    j[0] = (int)floor(f[0]);
                    j[1] = (int)floor(f[1]);
                    double val[2][2];
                    for (int i0 = 0; i0 < 2; ++i0)
                        for (int i1 = 0; i1 < 2; ++i1) {
                            int ia = j[0] + i0, ib = j[1] + i1;
                            double x = 0.0;
                            if (ia >= 0 && ia < G.n[ax[0]] && ib >= 0 && ib < G.n[ax[1]]) {
                                int idx[3];
                                idx[m] = l; idx[ax[0]] = ia; idx[ax[1]] = ib;
                                x = vol[((size_t)idx[2] * G.n[1] + idx[1]) * G.n[0] + idx[0]];
                            }
                            val[i0][i1] = x;
                        }
                    double w0 = f[0] - j[0], w1 = f[1] - j[1];
                    sum += (1 - w0) * (1 - w1) * val[0][0] + w0 * (1 - w1) * val[1][0] +
                           (1 - w0) * w1 * val[0][1] + w0 * w1 * val[1][1];
                    /* df/dp along each in-plane axis */
                    double dfd[2];
                    dfd[0] = ((1 - w1) * (val[1][0] - val[0][0]) + w1 * (val[1][1] - val[0][1])) / h;
                    dfd[1] = ((1 - w0) * (val[0][1] - val[0][0]) + w0 * (val[1][1] - val[1][0])) / h;
                    for (int c = 0; c < 2; ++c) {
                        int k = ax[c];
                        ds[k] += dfd[c] * (1.0 - t);
                        dq[k] += dfd[c] * t;
                        ds[m] += dfd[c] * D[k] * (t - 1.0) / D[m];
                        dq[m] += dfd[c] * (-D[k] * t / D[m]);
                    }
                }
                /* dL/dD */
                double dL[3];
                for (int k = 0; k < 3; ++k) dL[k] = h * D[k] / (len * fabs(D[m]));
                dL[m] -= h * len / (D[m] * fabs(D[m]));
                double ca = a - 0.5 * (nu - 1), cb = b - 0.5 * (nv - 1);
                for (int k = 0; k < 3; ++k) {
                    double dys = L * ds[k] - dL[k] * sum;
                    double dyq = L * dq[k] + dL[k] * sum;
                    acc[k] += gr * dys;
                    acc[3 + k] += gr * dyq;
                    acc[6 + k] += gr * ca * dyq;
                    acc[9 + k] += gr * cb * dyq;
                }
            }
        for (int k = 0; k < 12; ++k) dviews[(size_t)v * 12 + k] = acc[k];
    }
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the following calls (a timing aid; A^T's partial volumes are then summed in a
 * different grouping, so its result changes by rounding only). */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
