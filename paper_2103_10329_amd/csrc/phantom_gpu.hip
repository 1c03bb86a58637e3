// Synthetic phantoms on the device: exact line integrals through rotated
// ellipsoids and axis-aligned boxes (FP64), and supersampled voxel averages.
// Used to generate the learned preconditioner's training set on the GPU.
#include <hip/hip_runtime.h>

#include "mgct_internal.h"

namespace mgct {

// Parameter interval of segment s + t D (t in [0,1]) inside ellipsoid e.
__device__ __forceinline__ double chord_ellipsoid(const double *e, const double s[3], const double D[3]) {
    double sp[3], dp[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double ps = 0.0, pd = 0.0;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            ps += e[3 + r * 3 + k] * (s[r] - e[r]);
            pd += e[3 + r * 3 + k] * D[r];
        }
        sp[k] = ps / e[12 + k];
        dp[k] = pd / e[12 + k];
    }
    const double A = dp[0] * dp[0] + dp[1] * dp[1] + dp[2] * dp[2];
    const double B = 2.0 * (sp[0] * dp[0] + sp[1] * dp[1] + sp[2] * dp[2]);
    const double C = sp[0] * sp[0] + sp[1] * sp[1] + sp[2] * sp[2] - 1.0;
    const double disc = B * B - 4.0 * A * C;
    if (!(disc > 0.0) || !(A > 0.0)) return 0.0;
    const double r = sqrt(disc);
    const double t0 = fmax((-B - r) / (2.0 * A), 0.0), t1 = fmin((-B + r) / (2.0 * A), 1.0);
    return t1 > t0 ? t1 - t0 : 0.0;
}

__device__ __forceinline__ double chord_box(const double *bx, const double s[3], const double D[3]) {
    double t0 = 0.0, t1 = 1.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (D[k] == 0.0) {
            if (s[k] < bx[k] || s[k] > bx[3 + k]) return 0.0;
            continue;
        }
        double ta = (bx[k] - s[k]) / D[k], tb = (bx[3 + k] - s[k]) / D[k];
        if (ta > tb) { const double t = ta; ta = tb; tb = t; }
        t0 = fmax(t0, ta);
        t1 = fmin(t1, tb);
    }
    return t1 > t0 ? t1 - t0 : 0.0;
}

__global__ void k_synth_line_integrals(const double *__restrict__ views, int nviews, int nu, int nv,
                                       const double *__restrict__ ell, int K, const double *__restrict__ box, int J,
                                       float *__restrict__ out) {
    const long total = (long)nviews * nu * nv;
    for (long r = blockIdx.x * (long)blockDim.x + threadIdx.x; r < total; r += (long)gridDim.x * blockDim.x) {
        const int a = (int)(r % nu), b = (int)((r / nu) % nv), v = (int)(r / ((long)nu * nv));
        const double *g = views + (long)v * 12;
        const double ca = a - 0.5 * (nu - 1), cb = b - 0.5 * (nv - 1);
        double s[3], D[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            s[k] = g[k];
            D[k] = g[3 + k] + ca * g[6 + k] + cb * g[9 + k] - g[k];
        }
        const double len = sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
        double acc = 0.0;
        for (int e = 0; e < K; ++e) acc += ell[e * 16 + 15] * chord_ellipsoid(ell + e * 16, s, D);
        for (int e = 0; e < J; ++e) acc += box[e * 7 + 6] * chord_box(box + e * 7, s, D);
        out[r] = (float)(acc * len);
    }
}

__device__ __forceinline__ bool inside_ellipsoid(const double *e, const double p[3]) {
    double q = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double t = 0.0;
#pragma unroll
        for (int r = 0; r < 3; ++r) t += e[3 + r * 3 + k] * (p[r] - e[r]);
        t /= e[12 + k];
        q += t * t;
    }
    return q <= 1.0;
}

__global__ void k_synth_voxelize(int nx, int ny, int nz, double h, double ox, double oy, double oz,
                                 const double *__restrict__ ell, int K, const double *__restrict__ box, int J, int ss,
                                 float *__restrict__ vol) {
    const long n = (long)nx * ny * nz;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const int kx = (int)(i % nx), ky = (int)((i / nx) % ny), kz = (int)(i / ((long)nx * ny));
        const double c[3] = {ox + (kx - 0.5 * (nx - 1)) * h, oy + (ky - 0.5 * (ny - 1)) * h,
                             oz + (kz - 0.5 * (nz - 1)) * h};
        double acc = 0.0;
        const double inv = 1.0 / ((double)ss * ss * ss);
        for (int e = 0; e < K + J; ++e) {
            const bool is_e = e < K;
            const double *E = is_e ? ell + e * 16 : box + (e - K) * 7;
            // bounding-box rejection (voxel half-width h/2)
            bool far = false;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                double lo, hi;
                if (is_e) {
                    const double r = fmax(E[12], fmax(E[13], E[14]));
                    lo = E[k] - r;
                    hi = E[k] + r;
                } else {
                    lo = E[k];
                    hi = E[3 + k];
                }
                if (c[k] + 0.5 * h < lo || c[k] - 0.5 * h > hi) far = true;
            }
            if (far) continue;
            int cnt = 0;
            for (int sz = 0; sz < ss; ++sz)
                for (int sy = 0; sy < ss; ++sy)
                    for (int sx = 0; sx < ss; ++sx) {
                        const double p[3] = {c[0] + (-0.5 + (sx + 0.5) / ss) * h, c[1] + (-0.5 + (sy + 0.5) / ss) * h,
                                             c[2] + (-0.5 + (sz + 0.5) / ss) * h};
                        bool in;
                        if (is_e) in = inside_ellipsoid(E, p);
                        else in = p[0] >= E[0] && p[0] <= E[3] && p[1] >= E[1] && p[1] <= E[4] && p[2] >= E[2] &&
                                  p[2] <= E[5];
                        cnt += in;
                    }
            if (cnt) acc += (is_e ? E[15] : E[6]) * cnt * inv;
        }
        vol[i] = (float)acc;
    }
}

static unsigned grid_of(long n) {
    long g = (n + 255) / 256;
    if (g > 65535L * 8) g = 65535L * 8;
    return (unsigned)(g < 1 ? 1 : g);
}

hipError_t launch_synth_line_integrals(const double *views, int nviews, int nu, int nv, const double *ell, int K,
                                       const double *box, int J, float *out, hipStream_t s) {
    k_synth_line_integrals<<<grid_of((long)nviews * nu * nv), 256, 0, s>>>(views, nviews, nu, nv, ell, K, box, J, out);
    return hipGetLastError();
}

hipError_t launch_synth_voxelize(int nx, int ny, int nz, double h, const double *origin, const double *ell, int K,
                                 const double *box, int J, int ss, float *vol, hipStream_t s) {
    k_synth_voxelize<<<grid_of((long)nx * ny * nz), 256, 0, s>>>(nx, ny, nz, h, origin[0], origin[1], origin[2], ell, K,
                                                                 box, J, ss, vol);
    return hipGetLastError();
}

}  // namespace mgct
