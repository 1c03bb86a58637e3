// Streaming kernels around the projector: residual and norms, update and
// soft threshold, the 3^3 stencil and bilateral filters, grid transfers,
// and the OS-EMTR terms.  All are HBM-bound: one pass, coalesced along x.
#include <hip/hip_runtime.h>

#include "mgct_internal.h"

namespace mgct {

static inline unsigned grid_for(size_t n, int per_block = 256, unsigned cap = 65535u * 16u) {
    size_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

__global__ void k_fill(float *x, size_t n, float v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) x[i] = v;
}
hipError_t launch_fill(float *x, size_t n, float v, hipStream_t s) {
    k_fill<<<grid_for(n), 256, 0, s>>>(x, n, v);
    return hipGetLastError();
}

__global__ void k_copy(const float *x, float *y, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) y[i] = x[i];
}
hipError_t launch_copy(const float *x, float *y, size_t n, hipStream_t s) {
    k_copy<<<grid_for(n), 256, 0, s>>>(x, y, n);
    return hipGetLastError();
}

template <typename T> __device__ __forceinline__ float to_f(T v);
template <> __device__ __forceinline__ float to_f<float>(float v) { return v; }
template <> __device__ __forceinline__ float to_f<_Float16>(_Float16 v) { return (float)v; }
template <> __device__ __forceinline__ float to_f<uint16_t>(uint16_t v) { return __uint_as_float((uint32_t)v << 16); }

template <typename T>
__global__ void k_convert(const T *x, float *y, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = to_f<T>(x[i]);
}
hipError_t launch_convert_to_f32(const void *x, int dtype, float *y, size_t n, hipStream_t s) {
    if (dtype == MGCT_F32) k_convert<float><<<grid_for(n), 256, 0, s>>>((const float *)x, y, n);
    else if (dtype == MGCT_F16) k_convert<_Float16><<<grid_for(n), 256, 0, s>>>((const _Float16 *)x, y, n);
    else if (dtype == MGCT_BF16) k_convert<uint16_t><<<grid_for(n), 256, 0, s>>>((const uint16_t *)x, y, n);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

// Block-wide sum of one double per thread (256 threads).
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[256];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    return red[0];
}

// r = b - ax; partials[block] = sum of r^2 (of the stored r) over the
// block's grid-stride share.  b: F32/F16, ax and r: F32 or F16 storage.
template <typename TB, typename TA>
__global__ __launch_bounds__(256) void k_residual(const TB *b, const TA *ax, TA *r, size_t n, double *partials) {
    double acc = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const TA d = (TA)(to_f<TB>(b[i]) - to_f<TA>(ax[i]));
        r[i] = d;
        const double dd = (double)to_f<TA>(d);
        acc += dd * dd;
    }
    double t = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}
hipError_t launch_residual(const void *b, int b_dtype, const void *ax, void *r, int ax_dtype, size_t n,
                           double *partials, int nblocks, hipStream_t s) {
#define MGCT_RES(TB, TA) k_residual<TB, TA><<<nblocks, 256, 0, s>>>((const TB *)b, (const TA *)ax, (TA *)r, n, partials)
    if (b_dtype == MGCT_F32 && ax_dtype == MGCT_F32) MGCT_RES(float, float);
    else if (b_dtype == MGCT_F16 && ax_dtype == MGCT_F32) MGCT_RES(_Float16, float);
    else if (b_dtype == MGCT_F32 && ax_dtype == MGCT_F16) MGCT_RES(float, _Float16);
    else if (b_dtype == MGCT_F16 && ax_dtype == MGCT_F16) MGCT_RES(_Float16, _Float16);
    else return hipErrorInvalidValue;
#undef MGCT_RES
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_sumsq(const float *x, size_t n, double *partials) {
    double acc = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        acc += (double)x[i] * (double)x[i];
    double t = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}
hipError_t launch_sumsq(const float *x, size_t n, double *partials, int nblocks, hipStream_t s) {
    k_sumsq<<<nblocks, 256, 0, s>>>(x, n, partials);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_finish_sum(const double *partials, int n, double *out) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += partials[i];
    double t = block_sum(acc);
    if (threadIdx.x == 0) out[0] = t;
}
// Stage one of a wide sum: block b adds partials [b*per, (b+1)*per) in a fixed
// order into tmp[b].
__global__ __launch_bounds__(256) void k_sum_stage(const double *partials, int n, int per, double *tmp) {
    double acc = 0.0;
    const int beg = blockIdx.x * per, end = min(n, beg + per);
    for (int i = beg + threadIdx.x; i < end; i += 256) acc += partials[i];
    double t = block_sum(acc);
    if (threadIdx.x == 0) tmp[blockIdx.x] = t;
}
hipError_t launch_finish_sum(const double *partials, int n, double *out, hipStream_t s) {
    k_finish_sum<<<1, 256, 0, s>>>(partials, n, out);
    return hipGetLastError();
}
hipError_t launch_finish_sum_wide(const double *partials, int n, double *tmp, double *out, hipStream_t s) {
    if (n <= 4096) return launch_finish_sum(partials, n, out, s);
    const int nb = 256, per = (n + nb - 1) / nb;
    k_sum_stage<<<nb, 256, 0, s>>>(partials, n, per, tmp);
    k_finish_sum<<<1, 256, 0, s>>>(tmp, nb, out);
    return hipGetLastError();
}

// Stage one of the sum over a view subset: block b takes the (view, row tile)
// entries [b*per, (b+1)*per) in order and adds the n_ct partials of those
// whose view is a multiple of step.
__global__ __launch_bounds__(256) void k_sum_stage_views(const double *partials, const int *order, int n_ct, int n_t,
                                                         int n_rt, int step, int per, double *tmp) {
    double acc = 0.0;
    const int beg = blockIdx.x * per, end = min(n_t, beg + per);
    for (int t = beg; t < end; ++t) {
        if ((order[t] / n_rt) % step) continue;  // block-uniform
        for (int ct = threadIdx.x; ct < n_ct; ct += 256) acc += partials[(long)t * n_ct + ct];
    }
    double r = block_sum(acc);
    if (threadIdx.x == 0) tmp[blockIdx.x] = r;
}
hipError_t launch_finish_sum_views(const double *partials, const int *order, int n_ct, int n_t, int n_rt, int step,
                                   double *tmp, double *out, hipStream_t s) {
    const int nb = 256, per = (n_t + nb - 1) / nb;
    k_sum_stage_views<<<nb, 256, 0, s>>>(partials, order, n_ct, n_t, n_rt, step, per, tmp);
    k_finish_sum<<<1, 256, 0, s>>>(tmp, nb, out);
    return hipGetLastError();
}

__global__ void k_axpy(float *y, const float *x, float alpha, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = fmaf(alpha, x[i], y[i]);
}
hipError_t launch_axpy(float *y, const float *x, double alpha, size_t n, hipStream_t s) {
    k_axpy<<<grid_for(n), 256, 0, s>>>(y, x, (float)alpha, n);
    return hipGetLastError();
}

__global__ void k_scale(const float *x, float *y, float a, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = a * x[i];
}
hipError_t launch_scale(const float *x, float *y, float a, size_t n, hipStream_t s) {
    k_scale<<<grid_for(n), 256, 0, s>>>(x, y, a, n);
    return hipGetLastError();
}

__global__ void k_add(const float *x, const float *y, float *out, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = x[i] + y[i];
}
hipError_t launch_add(const float *x, const float *y, float *out, size_t n, hipStream_t s) {
    k_add<<<grid_for(n), 256, 0, s>>>(x, y, out, n);
    return hipGetLastError();
}

// Learned step's judge: keep mu_try if its squared residual r1 is below the
// current one r0, else take the plain update mu + u.  counters[0/1] count
// accepted / rejected steps.
__global__ void k_select_update(float *mu, const float *u, const float *mu_try, size_t n, const double *r0,
                                const double *r1, unsigned *counters) {
    const bool keep = r1[0] < r0[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(counters + (keep ? 0 : 1), 1u);
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        mu[i] = keep ? mu_try[i] : mu[i] + u[i];
}
hipError_t launch_select_update(float *mu, const float *u, const float *mu_try, size_t n, const double *r0,
                                const double *r1, unsigned *counters, hipStream_t s) {
    k_select_update<<<grid_for(n), 256, 0, s>>>(mu, u, mu_try, n, r0, r1, counters);
    return hipGetLastError();
}

// x *= 1/sqrt(sumsq[0]); lambda_out[0] = sqrt(sumsq[0]) (power iteration).
__global__ void k_scale_inv_sqrt(float *x, size_t n, const double *sumsq, double *lambda_out) {
    const double nrm = sqrt(sumsq[0]);
    const float inv = nrm > 0.0 ? (float)(1.0 / nrm) : 0.f;
    if (blockIdx.x == 0 && threadIdx.x == 0 && lambda_out) lambda_out[0] = nrm;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        x[i] *= inv;
}
hipError_t launch_scale_by_inv_sqrt(float *x, size_t n, const double *sumsq, double *lambda_out, hipStream_t s) {
    k_scale_inv_sqrt<<<grid_for(n), 256, 0, s>>>(x, n, sumsq, lambda_out);
    return hipGetLastError();
}

__global__ void k_soft(float *x, size_t n, float lam) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        float v = x[i];
        float m = fmaxf(fabsf(v) - lam, 0.f);
        x[i] = copysignf(m, v);
    }
}
hipError_t launch_soft_threshold(float *x, size_t n, float lam, hipStream_t s) {
    k_soft<<<grid_for(n), 256, 0, s>>>(x, n, lam);
    return hipGetLastError();
}

// Circular 3^3 convolution: out[z,y,x] = sum taps[d] in[(z,y,x) - d].
__global__ __launch_bounds__(256) void k_stencil27(const float *in, float *out, int nx, int ny, int nz,
                                                   const float *__restrict__ taps) {
    const size_t n = (size_t)nx * ny * nz;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x) {
        int x, y, z;
        split3(idx, nx, ny, x, y, z);
        // FP64 accumulation: a zero-DC kernel applied to a smooth field is a
        // difference of nearly equal sums, so FP32 would lose digits here.
        double acc = 0.0;
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz) {
            const int zz = (z - dz + nz) % nz;
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy) {
                const int yy = (y - dy + ny) % ny;
                const float *row = in + ((size_t)zz * ny + yy) * nx;
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const float w = taps[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)];
                    const int xx = (x - dx + nx) % nx;
                    acc = fma((double)w, (double)row[xx], acc);
                }
            }
        }
        out[idx] = (float)acc;
    }
}
hipError_t launch_stencil27(const float *in, float *out, int nx, int ny, int nz, const float *taps, hipStream_t s) {
    k_stencil27<<<grid_for((size_t)nx * ny * nz), 256, 0, s>>>(in, out, nx, ny, nz, taps);
    return hipGetLastError();
}

// 3^3 bilateral filter, in-grid neighbours only, normalised.
// 3^3 bilateral filter: neighbours inside the grid, weight
// exp(-|offset|^2 / (2 sigma_s^2) - (v - c)^2 / (2 sigma_r^2)).  All 27 taps are
// unrolled with the outside ones masked to weight 0 (adding exact zeros keeps
// the sums of the branching form), 32-bit indices (grids hold fewer than
// 2^31 voxels) and the hardware exponential (about 1e-7 relative here).
__global__ __launch_bounds__(256) void k_bilateral(const float *__restrict__ in, float *__restrict__ out, int nx,
                                                   int ny, int nz, float inv2ss, float inv2sr) {
    const long n = (long)nx * ny * nz;
    // the loop counter is 64-bit (counter + stride may pass 2^31); the voxel
    // index itself fits 32 bits
    for (long li = blockIdx.x * (long)blockDim.x + threadIdx.x; li < n; li += (long)gridDim.x * blockDim.x) {
        const int idx = (int)li;
        int x, y, z;
        split3(li, nx, ny, x, y, z);
        const float c = in[idx];
        float num = 0.f, den = 0.f;
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const bool ok = (unsigned)(x + dx) < (unsigned)nx && (unsigned)(y + dy) < (unsigned)ny &&
                                    (unsigned)(z + dz) < (unsigned)nz;
                    const float v = in[ok ? idx + (dz * ny + dy) * nx + dx : idx];
                    const float d = v - c;
                    const float w = ok ? __expf(-(float)(dx * dx + dy * dy + dz * dz) * inv2ss - d * d * inv2sr) : 0.f;
                    num = fmaf(w, v, num);
                    den += w;
                }
        out[idx] = num / den;
    }
}
hipError_t launch_bilateral(const float *in, float *out, int nx, int ny, int nz, float sigma_s, float sigma_r,
                            hipStream_t s) {
    float inv2ss = 1.f / (2.f * sigma_s * sigma_s), inv2sr = 1.f / (2.f * sigma_r * sigma_r);
    k_bilateral<<<grid_for((size_t)nx * ny * nz), 256, 0, s>>>(in, out, nx, ny, nz, inv2ss, inv2sr);
    return hipGetLastError();
}

// coarse = 2x2x2 block mean; sizes are the fine grid's.
__global__ void k_restrict_vol(const float *f, float *c, int nx, int ny, int nz) {
    const int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    const size_t n = (size_t)cx * cy * cz;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x) {
        int x, y, z;
        split3(idx, cx, cy, x, y, z);
        float acc = 0.f;
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy) {
                const float *r = f + ((size_t)(2 * z + dz) * ny + (2 * y + dy)) * nx + 2 * x;
                acc += r[0] + r[1];
            }
        c[idx] = acc * 0.125f;
    }
}
hipError_t launch_restrict_volume(const float *fine, float *coarse, int nx, int ny, int nz, hipStream_t s) {
    k_restrict_vol<<<grid_for((size_t)nx * ny * nz / 8), 256, 0, s>>>(fine, coarse, nx, ny, nz);
    return hipGetLastError();
}

// coarse stack = 2x2 pixel mean; sizes are the fine grid's.
__global__ void k_restrict_stack(const float *f, float *c, int nviews, int nv, int nu) {
    const int cu = nu / 2, cv = nv / 2;
    const size_t n = (size_t)nviews * cu * cv;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x) {
        int a, b, v;
        split3(idx, cu, cv, a, b, v);
        const float *r0 = f + ((size_t)v * nv + 2 * b) * nu + 2 * a;
        const float *r1 = r0 + nu;
        c[idx] = 0.25f * ((r0[0] + r0[1]) + (r1[0] + r1[1]));
    }
}
hipError_t launch_restrict_stack(const float *fine, float *coarse, int nviews, int nv, int nu, hipStream_t s) {
    k_restrict_stack<<<grid_for((size_t)nviews * nv * nu / 4), 256, 0, s>>>(fine, coarse, nviews, nv, nu);
    return hipGetLastError();
}

// fine += trilinear cell-centred prolongation of (cnew - cold); fine sizes given.
__device__ __forceinline__ void prolong_taps(int i, int nc, int &i0, int &i1, float &w1) {
    // fine cell i sits at coarse coordinate (i + 1/2)/2 - 1/2 = i/2 - 1/4
    const int m = i >> 1;
    if (i & 1) { i0 = m; i1 = min(m + 1, nc - 1); }
    else       { i0 = max(m - 1, 0); i1 = m; }
    w1 = (i & 1) ? 0.25f : 0.75f;  // weight of i1
}
__global__ void k_prolong_add(const float *cn, const float *co, float *f, int nx, int ny, int nz) {
    const int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    const size_t n = (size_t)nx * ny * nz;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x) {
        int x, y, z;
        split3(idx, nx, ny, x, y, z);
        int x0, x1, y0, y1, z0, z1;
        float wx, wy, wz;
        prolong_taps(x, cx, x0, x1, wx);
        prolong_taps(y, cy, y0, y1, wy);
        prolong_taps(z, cz, z0, z1, wz);
        auto d = [&](int zz, int yy, int xx) {
            const size_t o = ((size_t)zz * cy + yy) * cx + xx;
            return cn[o] - co[o];
        };
        const float c00 = d(z0, y0, x0) + wx * (d(z0, y0, x1) - d(z0, y0, x0));
        const float c01 = d(z0, y1, x0) + wx * (d(z0, y1, x1) - d(z0, y1, x0));
        const float c10 = d(z1, y0, x0) + wx * (d(z1, y0, x1) - d(z1, y0, x0));
        const float c11 = d(z1, y1, x0) + wx * (d(z1, y1, x1) - d(z1, y1, x0));
        const float c0 = c00 + wy * (c01 - c00), c1 = c10 + wy * (c11 - c10);
        f[idx] += c0 + wz * (c1 - c0);
    }
}
hipError_t launch_prolong_add(const float *cnew, const float *cold, float *fine, int nx, int ny, int nz,
                              hipStream_t s) {
    k_prolong_add<<<grid_for((size_t)nx * ny * nz), 256, 0, s>>>(cnew, cold, fine, nx, ny, nz);
    return hipGetLastError();
}

// OS-EMTR terms for the views of one subset: e = exp(-l),
// num_src = e - exp(-b), den_src = e * (A 1).
// OS-EMTR: num and den from the back-projector's view-chunk partials
// (summed in FP64 in chunk order; nchunks <= 1: num/den already final) and
// the max of den, folded into *maxbits with an ordered-integer atomic max
// (den >= 0, so its bit pattern orders like its value).
__global__ __launch_bounds__(256) void k_emtr_reduce(const float *__restrict__ part_num,
                                                     const float *__restrict__ part_den, float *__restrict__ num,
                                                     float *__restrict__ den, size_t n, int nchunks,
                                                     unsigned *maxbits) {
    float acc = 0.f;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        float d;
        if (nchunks > 1) {
            double sn = 0.0, sd = 0.0;
            for (int c = 0; c < nchunks; ++c) {
                sn += (double)part_num[c * n + i];
                sd += (double)part_den[c * n + i];
            }
            num[i] = (float)sn;
            d = (float)sd;
            den[i] = d;
        } else {
            d = den[i];
        }
        acc = fmaxf(acc, d);
    }
    __shared__ float red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(maxbits, __float_as_uint(fmaxf(red[0], 0.f)));
}
hipError_t launch_emtr_reduce(const float *part_num, const float *part_den, float *num, float *den, size_t n,
                              int nchunks, unsigned *maxbits, hipStream_t s) {
    k_emtr_reduce<<<grid_for(n, 256, 1024), 256, 0, s>>>(part_num, part_den, num, den, n, nchunks, maxbits);
    return hipGetLastError();
}

// vol += num/den where den > 1e-6 * max(den).
__global__ void k_emtr_update(float *vol, const float *num, const float *den, size_t n, const unsigned *maxbits) {
    const float thr = 1e-6f * __uint_as_float(maxbits[0]);
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float d = den[i];
        if (d > thr) vol[i] += num[i] / d;
    }
}
hipError_t launch_emtr_update(float *vol, const float *num, const float *den, size_t n, unsigned *maxbits,
                              hipStream_t s) {
    k_emtr_update<<<grid_for(n), 256, 0, s>>>(vol, num, den, n, maxbits);
    return hipGetLastError();
}

// x[k] = SplitMix64 uniform: state seed + (k+1) * 0x9E3779B97F4A7C15, top 53 bits / 2^53.
__global__ void k_splitmix(float *x, size_t n, uint64_t seed) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z = z ^ (z >> 31);
        x[i] = (float)((double)(z >> 11) * (1.0 / 9007199254740992.0));
    }
}
hipError_t launch_splitmix_uniform(float *x, size_t n, uint64_t seed, hipStream_t s) {
    k_splitmix<<<grid_for(n), 256, 0, s>>>(x, n, seed);
    return hipGetLastError();
}

}  // namespace mgct

namespace mgct {

// Content key of an array of 32-bit words: the sum, modulo 2^64, of the
// SplitMix64 finaliser applied to (word + (i+1) * golden ratio) over all
// words i.  The sum is order-independent, so the blocks' partial sums may
// be combined in any order; used to tell apart filter arrays that sit at the
// same address.
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_hash_words(const uint32_t *__restrict__ x, size_t n,
                                                    unsigned long long *__restrict__ partials) {
    unsigned long long acc = 0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        acc += mix64((unsigned long long)x[i] + (unsigned long long)(i + 1) * 0x9E3779B97F4A7C15ull);
    __shared__ unsigned long long s[256];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = s[0];
}

__global__ void k_hash_finish(const unsigned long long *__restrict__ partials, int n, unsigned long long *out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        unsigned long long t = 0;
        for (int i = 0; i < n; ++i) t += partials[i];
        out[0] = t;
    }
}

hipError_t launch_hash_words(const void *x, size_t n_words, unsigned long long *partials, int nblocks,
                             unsigned long long *out, hipStream_t s) {
    k_hash_words<<<nblocks, 256, 0, s>>>((const uint32_t *)x, n_words, partials);
    k_hash_finish<<<1, 64, 0, s>>>(partials, nblocks, out);
    return hipGetLastError();
}

}  // namespace mgct
