// Joseph cone-beam projector A and its transpose A^T for gfx950.
//
// Forward (ray-driven): one lane per detector pixel, lanes of a wavefront
// are 64 consecutive detector rows of one column.  The volume is first copied
// into a zero-padded, z-fastest layout vt[x][y][z], so that for the x- and
// y-major rays of a column (whose z coordinate at a plane grows with the
// row) the two bilinear taps along z are adjacent and the 64 lanes of a wave
// touch a few contiguous cache lines per plane.  Sampling positions are
// affine in the plane index; the per-ray set-up (plane range, slopes, the
// spacing factor h|D|/|D_m|) is done in FP64, the sampling loop in FP32.
//
// Transpose (voxel-driven gather, no atomics): one lane per voxel, lanes of a
// wavefront are consecutive z of one (x, y) column.  For the geometry in
// which the detector columns are horizontal and the rows vertical, the
// detector column hit by a ray through (x, y, .) does not depend on z, so
// the candidate columns of every view are wave-uniform (scalar loop, scalar
// loads of the per-column table); each lane then walks only the handful of
// rows whose sample on the voxel's plane lies within one voxel of it in z.
// The data are first scaled by each ray's spacing factor and transposed to
// [view][column][row] so that those row reads are contiguous across lanes.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mgct_internal.h"

namespace mgct {

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
    u += 0x7fffu + ((u >> 16) & 1u);                     // round to nearest even
    return (uint16_t)(u >> 16);
}

template <typename T> __device__ __forceinline__ float load_f(const T *p, long i);
template <> __device__ __forceinline__ float load_f<float>(const float *p, long i) { return p[i]; }
template <> __device__ __forceinline__ float load_f<uint16_t>(const uint16_t *p, long i) { return bf16_to_f32(p[i]); }
template <> __device__ __forceinline__ float load_f<_Float16>(const _Float16 *p, long i) { return (float)p[i]; }

// Load element `i` of an array smaller than 4 GiB through a 32-bit byte
// offset, so that the access can use the scalar-base + 32-bit-offset form.
template <typename T> __device__ __forceinline__ float load_off(const T *p, uint32_t i) {
    const uint32_t byte = i * (uint32_t)sizeof(T);
    return load_f(reinterpret_cast<const T *>(reinterpret_cast<const char *>(p) + byte), 0);
}

// Elements i and i+1 through a 32-bit byte offset, as one access.
__device__ __forceinline__ float2 load_pair(const float *p, uint32_t i) {
    const char *q = reinterpret_cast<const char *>(p) + i * 4u;
    float2 r;
    __builtin_memcpy(&r, __builtin_assume_aligned(q, 4), 8);
    return r;
}
__device__ __forceinline__ float2 load_pair(const uint16_t *p, uint32_t i) {
    const char *q = reinterpret_cast<const char *>(p) + i * 2u;
    uint32_t u;
    __builtin_memcpy(&u, __builtin_assume_aligned(q, 2), 4);
    return make_float2(__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u));
}

// Elements i .. i+3 through a 32-bit byte offset, as one access.
__device__ __forceinline__ float4 load_quad(const float *p, uint32_t i) {
    const char *q = reinterpret_cast<const char *>(p) + i * 4u;
    float4 r;
    __builtin_memcpy(&r, __builtin_assume_aligned(q, 4), 16);
    return r;
}
__device__ __forceinline__ float4 load_quad(const _Float16 *p, uint32_t i) {
    const char *q = reinterpret_cast<const char *>(p) + i * 2u;
    _Float16 h[4];
    __builtin_memcpy(h, __builtin_assume_aligned(q, 2), 8);
    return make_float4((float)h[0], (float)h[1], (float)h[2], (float)h[3]);
}

template <typename T> __device__ __forceinline__ void store_f(T *p, long i, float x);
template <> __device__ __forceinline__ void store_f<float>(float *p, long i, float x) { p[i] = x; }
template <> __device__ __forceinline__ void store_f<uint16_t>(uint16_t *p, long i, float x) { p[i] = f32_to_bf16(x); }
template <> __device__ __forceinline__ void store_f<_Float16>(_Float16 *p, long i, float x) { p[i] = (_Float16)x; }
// Two consecutive values at even index i in one 8-byte (float) or 4-byte
// (bf16) store.
template <typename T> __device__ __forceinline__ void store_pair(T *p, long i, float x0, float x1);
template <> __device__ __forceinline__ void store_pair<float>(float *p, long i, float x0, float x1) {
    *reinterpret_cast<float2 *>(p + i) = make_float2(x0, x1);
}
template <> __device__ __forceinline__ void store_pair<uint16_t>(uint16_t *p, long i, float x0, float x1) {
    *reinterpret_cast<uint32_t *>(p + i) = (uint32_t)f32_to_bf16(x0) | ((uint32_t)f32_to_bf16(x1) << 16);
}

// ---------------------------------------------------------------- set-up --

// Spacing factor h |D| / |D_m| of ray (a, b) of view V and its direction D
// (voxel-index units).  Shared by the projector and the data pre-scaling of
// the transpose so that both use bit-identical factors.
__device__ __forceinline__ double ray_setup(const ViewIdx &V, int nu, int nv, int a, int b, double D[3]) {
    double ca = a - 0.5 * (nu - 1), cb = b - 0.5 * (nv - 1);
#pragma unroll
    for (int k = 0; k < 3; ++k) D[k] = (V.d[k] + ca * V.u[k] + cb * V.v[k]) - V.s[k];
    return sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
}

// Restrict [lo, hi] to the planes l with A + l*B inside [bmin, bmax].
// A fraction in [0, 1) as a 0.32 fixed-point value (rounded, kept below 1).
__device__ __forceinline__ uint32_t frac_u32(double f) {
    return (uint32_t)fmin(rint(f * 4294967296.0), 4294967295.0);
}

__device__ __forceinline__ void clip_range(double &lo, double &hi, double A, double B, double bmin, double bmax) {
    if (B > 0.0) {
        lo = fmax(lo, ceil((bmin - A) / B));
        hi = fmin(hi, floor((bmax - A) / B));
    } else if (B < 0.0) {
        lo = fmax(lo, ceil((bmax - A) / B));
        hi = fmin(hi, floor((bmin - A) / B));
    } else if (A < bmin || A > bmax) {
        hi = lo - 1.0;
    }
}

// ------------------------------------------------------ volume transpose --

// vol[z][y][x] -> vt[x+P][y+P][z+P] (P = kVolPad); the padding stays zero.
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_transpose_volume(const TI *__restrict__ vol, TO *__restrict__ vt, int nx,
                                                          int ny, int nz) {
    __shared__ float tile[64][65];
    const int x0 = blockIdx.x * 64, z0 = blockIdx.y * 64, y = blockIdx.z;
    const int t = threadIdx.x;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        int zl = (t >> 6) + 4 * r, xl = t & 63;
        int z = z0 + zl, x = x0 + xl;
        float v = 0.f;
        if (z < nz && x < nx) v = load_f(vol, ((long)z * ny + y) * nx + x);
        tile[zl][xl] = v;
    }
    __syncthreads();
    const long PY = ny + 2 * kVolPad, PZ = nz + 2 * kVolPad;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        int xl = (t >> 6) + 4 * r, zl = t & 63;
        int z = z0 + zl, x = x0 + xl;
        if (z < nz && x < nx) store_f(vt, ((long)(x + kVolPad) * PY + (y + kVolPad)) * PZ + (z + kVolPad), tile[zl][xl]);
    }
}

hipError_t launch_transpose_volume(const void *vol, int vol_dtype, void *vt, int vt_dtype, const Level &L,
                                   hipStream_t s) {
    dim3 grid((L.nx + 63) / 64, (L.nz + 63) / 64, L.ny);
    if (vol_dtype == MGCT_F32 && vt_dtype == MGCT_F32)
        k_transpose_volume<float, float><<<grid, 256, 0, s>>>((const float *)vol, (float *)vt, L.nx, L.ny, L.nz);
    else if (vol_dtype == MGCT_BF16 && vt_dtype == MGCT_BF16)
        k_transpose_volume<uint16_t, uint16_t>
            <<<grid, 256, 0, s>>>((const uint16_t *)vol, (uint16_t *)vt, L.nx, L.ny, L.nz);
    else if (vol_dtype == MGCT_F32 && vt_dtype == MGCT_BF16)
        k_transpose_volume<float, uint16_t><<<grid, 256, 0, s>>>((const float *)vol, (uint16_t *)vt, L.nx, L.ny, L.nz);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// ----------------------------------------------- pair-expanded copies --
//
// For the separable projector every Joseph sample needs the 2x2 taps
// (in-plane a, z) at (a0, z0) .. (a0+1, z0+1).  Two copies store each voxel
// next to its neighbour along a: vtx[x][y][z] = (mu[x][y][z], mu[x][y+1][z])
// for x-major rays (a = y) and vty[y][x][z] = (mu[x][y][z], mu[x+1][y][z])
// for y-major rays (a = x), zero-padded by kVolPad, z fastest.  The four
// taps of a sample are then 4 consecutive values: one 16-byte gather.
// Grid: (x tiles of TX, z tiles of 64, y + 1 for y in [-1, ny-1]); each
// pair leaves in one store.
template <typename TI, typename TO, int TX>
__global__ __launch_bounds__(256) void k_transpose_pairs(const TI *__restrict__ vol, TO *__restrict__ vtx,
                                                         TO *__restrict__ vty, int nx, int ny, int nz) {
    __shared__ float t0[64][TX + 3];  // row y, x in [x0-1, x0+TX]
    __shared__ float t1[64][TX + 1];  // row y+1, x in [x0, x0+TX-1]
    const int x0 = blockIdx.x * TX, z0 = blockIdx.y * 64, y = (int)blockIdx.z - 1;
    const int t = threadIdx.x;
    for (int q = t; q < 64 * (TX + 2); q += 256) {
        const int zl = q / (TX + 2), xl = q % (TX + 2);
        const int z = z0 + zl, x = x0 - 1 + xl;
        float v = 0.f;
        if (y >= 0 && z < nz && x >= 0 && x < nx) v = load_f(vol, ((long)z * ny + y) * nx + x);
        t0[zl][xl] = v;
    }
    for (int q = t; q < 64 * TX; q += 256) {
        const int zl = q / TX, xl = q % TX;
        const int z = z0 + zl, x = x0 + xl;
        float v = 0.f;
        if (y + 1 < ny && z < nz && x < nx) v = load_f(vol, ((long)z * ny + (y + 1)) * nx + x);
        t1[zl][xl] = v;
    }
    __syncthreads();
    const long PX = nx + 2 * kVolPad, PY = ny + 2 * kVolPad, PZ = nz + 2 * kVolPad;
    // vtx pairs along y: x in [x0, x0+TX-1], y in [-1, ny-1]
    for (int q = t; q < TX * 64; q += 256) {
        const int xl = q >> 6, zl = q & 63;
        const int z = z0 + zl, x = x0 + xl;
        if (z < nz && x < nx) {
            const long o = (((long)(x + kVolPad) * PY + (y + kVolPad)) * PZ + (z + kVolPad)) * 2;
            store_pair(vtx, o, t0[zl][xl + 1], t1[zl][xl]);
        }
    }
    // vty pairs along x: y in [0, ny-1], x in [x0, x0+TX-1] (and x = -1 for the first tile)
    if (y >= 0) {
        for (int q = t; q < (TX + 1) * 64; q += 256) {
            const int xl = (q >> 6) - 1, zl = q & 63;
            const int z = z0 + zl, x = x0 + xl;
            if (z < nz && x < nx && (xl >= 0 || x0 == 0)) {
                const long o = (((long)(y + kVolPad) * PX + (x + kVolPad)) * PZ + (z + kVolPad)) * 2;
                store_pair(vty, o, t0[zl][xl + 1], t0[zl][xl + 2]);
            }
        }
    }
}

// OS-EMTR update mu += num/den where den > 1e-6 max(den) (eq. 3), also
// writing each new value into the pair copies so the next subset's
// projection needs no fresh transposition.  Voxel (x, y, z) sits in vtx pair
// (x, y) first and (x, y-1) second, and in vty pair (y, x) first and
// (y, x-1) second (pairs exist from -1, so every neighbour is in range).
template <typename TO>
__global__ void k_emtr_update_pairs(float *__restrict__ vol, const float *__restrict__ num,
                                    const float *__restrict__ den, const unsigned *__restrict__ maxbits,
                                    TO *__restrict__ vtx, TO *__restrict__ vty, int nx, int ny, int nz) {
    const float thr = 1e-6f * __uint_as_float(maxbits[0]);
    const size_t n = (size_t)nx * ny * nz;
    const long PX = nx + 2 * kVolPad, PY = ny + 2 * kVolPad, PZ = nz + 2 * kVolPad;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        float m = vol[i];
        const float d = den[i];
        if (d > thr) {
            m += num[i] / d;
            vol[i] = m;
        }
        int x, y, z;
        split3(i, nx, ny, x, y, z);
        const long ox = (((long)(x + kVolPad) * PY + (y + kVolPad)) * PZ + (z + kVolPad)) * 2;
        store_f(vtx, ox, m);
        store_f(vtx, ox - 2 * PZ + 1, m);
        const long oy = (((long)(y + kVolPad) * PX + (x + kVolPad)) * PZ + (z + kVolPad)) * 2;
        store_f(vty, oy, m);
        store_f(vty, oy - 2 * PZ + 1, m);
    }
}

hipError_t launch_emtr_update_pairs(float *vol, const float *num, const float *den, const unsigned *maxbits,
                                    void *vtx, void *vty, int vt_dtype, const Level &L, hipStream_t s) {
    const size_t n = L.vox();
    const unsigned g = (unsigned)std::min<size_t>((n + 255) / 256, 65535);
    if (vt_dtype == MGCT_F32)
        k_emtr_update_pairs<float><<<g, 256, 0, s>>>(vol, num, den, maxbits, (float *)vtx, (float *)vty, L.nx, L.ny,
                                                     L.nz);
    else if (vt_dtype == MGCT_BF16)
        k_emtr_update_pairs<uint16_t><<<g, 256, 0, s>>>(vol, num, den, maxbits, (uint16_t *)vtx, (uint16_t *)vty,
                                                        L.nx, L.ny, L.nz);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

#ifndef MGCT_TP_X
#define MGCT_TP_X 16
#endif
constexpr int kTpX = MGCT_TP_X;  // x tile width of the pair-copy transposition

hipError_t launch_transpose_pairs(const void *vol, int vol_dtype, void *vtx, void *vty, int vt_dtype, const Level &L,
                                  hipStream_t s) {
    dim3 grid((L.nx + kTpX - 1) / kTpX, (L.nz + 63) / 64, L.ny + 1);
#define MGCT_TP(TI, TO) \
    k_transpose_pairs<TI, TO, kTpX><<<grid, 256, 0, s>>>((const TI *)vol, (TO *)vtx, (TO *)vty, L.nx, L.ny, L.nz)
    if (vol_dtype == MGCT_F32 && vt_dtype == MGCT_F32) MGCT_TP(float, float);
    else if (vol_dtype == MGCT_BF16 && vt_dtype == MGCT_BF16) MGCT_TP(uint16_t, uint16_t);
    else if (vol_dtype == MGCT_F32 && vt_dtype == MGCT_BF16) MGCT_TP(float, uint16_t);
    else return hipErrorInvalidValue;
#undef MGCT_TP
    return hipGetLastError();
}

size_t pair_copy_elems(const Level &L) {
    return (size_t)(L.nx + 2 * kVolPad) * (L.ny + 2 * kVolPad) * (L.nz + 2 * kVolPad) * 2;
}

__device__ __forceinline__ float4 load_quad(const uint16_t *p, uint32_t i) {
    const char *q = reinterpret_cast<const char *>(p) + i * 2u;
    uint2 u;
    __builtin_memcpy(&u, __builtin_assume_aligned(q, 4), 8);
    return make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u), __uint_as_float(u.y << 16),
                       __uint_as_float(u.y & 0xffff0000u));
}

// ------------------------------------------------------------- projector --

template <typename VT, typename PT>
__global__ __launch_bounds__(256) void k_project(const VT *__restrict__ vt, PT *__restrict__ proj,
                                                 const ViewIdx *__restrict__ views, const uint8_t *__restrict__ axis,
                                                 long axis_view_stride, long axis_row_stride, int nx, int ny, int nz,
                                                 int nu, int nv, double h, int view0, int view_step) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int a = blockIdx.x * 4 + w;
    const int b = blockIdx.y * 64 + lane;
    const int vl = blockIdx.z;
    const int v = view0 + vl * view_step;
    if (a >= nu || b >= nv) return;  // no barrier below

    const ViewIdx &V = views[v];
    double D[3];
    const double len = ray_setup(V, nu, nv, a, b, D);
    const int m = axis[v * axis_view_stride + b * axis_row_stride + a];  // 0: x-major, 1: y-major
    const int ia = (m == 0) ? 1 : 0;
    const double Dm = D[m], Da = D[ia], Dz = D[2];
    const double sm = V.s[m], sa = V.s[ia], sz = V.s[2];
    // sample on plane l: (in-plane a, z) = (Aa + l Ba, Az + l Bz)
    const double Ba = Da / Dm, Bz = Dz / Dm;
    const double Aa = sa - sm * Ba, Az = sz - sm * Bz;
    const int n_m = (m == 0) ? nx : ny, n_a = (m == 0) ? ny : nx;
    // planes between source (t = 0) and pixel (t = 1)
    double lo = fmax(0.0, ceil(fmin(sm, sm + Dm)));
    double hi = fmin((double)(n_m - 1), floor(fmax(sm, sm + Dm)));
    // samples whose bilinear footprint can touch the grid, with half a voxel
    // of margin inside the 2-voxel zero padding
    clip_range(lo, hi, Aa, Ba, -1.5, n_a + 0.5);
    clip_range(lo, hi, Az, Bz, -1.5, nz + 0.5);
    // a degenerate ray (pixel at the source) contributes nothing
    if (!(fabs(Dm) > 0.0) || !isfinite(Aa) || !isfinite(Az) || !isfinite(Ba) || !isfinite(Bz)) hi = lo - 1.0;
    const float scale = (float)(h * len / fabs(Dm));

    float acc = 0.f;
    if (lo <= hi) {
        const int l0 = (int)lo, l1 = (int)hi;
        const int PY = ny + 2 * kVolPad, PZ = nz + 2 * kVolPad;
        const int Sm = (m == 0) ? PY * PZ : PZ;
        const int Sa = (m == 0) ? PZ : PY * PZ;
        // The sample's padded in-plane and z coordinates are linear in the
        // plane index; both step from plane l0 in 32.32 fixed point (integer
        // part = lower tap, fraction = its weight): integer adds with carry
        // per plane instead of FP64 arithmetic, which issues at half the FP32
        // rate here.  Starts and slopes are rounded once from FP64; the drift
        // stays below 2^-33 per plane, far below the FP32 rounding of the
        // weights.  The clipped range keeps every sample at least half a voxel
        // inside the padded copy.
        const double fa0 = fma((double)l0, Ba, Aa + kVolPad), fz0 = fma((double)l0, Bz, Az + kVolPad);
        const double ga0 = floor(fa0), gz0 = floor(fz0), gba = floor(Ba), gbz = floor(Bz);
        int ai = (int)ga0, zi = (int)gz0;
        uint32_t af = frac_u32(fa0 - ga0), zf = frac_u32(fz0 - gz0);
        const int bai = (int)gba, bzi = (int)gbz;
        const uint32_t baf = frac_u32(Ba - gba), bzf = frac_u32(Bz - gbz);
        int off_m = (l0 + kVolPad) * Sm;
        for (int l = l0; l <= l1; ++l, off_m += Sm) {
            const float wa = (float)af * 0x1p-32f, wz = (float)zf * 0x1p-32f;
            const int off = off_m + ai * Sa + zi;
            const float p00 = load_f(vt, off), p01 = load_f(vt, off + 1);
            const float p10 = load_f(vt, off + Sa), p11 = load_f(vt, off + Sa + 1);
            const float q0 = fmaf(wz, p01 - p00, p00), q1 = fmaf(wz, p11 - p10, p10);
            acc += fmaf(wa, q1 - q0, q0);
            const uint32_t na = af + baf, nz2 = zf + bzf;
            ai += bai + (na < af ? 1 : 0);
            zi += bzi + (nz2 < zf ? 1 : 0);
            af = na;
            zf = nz2;
        }
    }
    store_f(proj, ((long)vl * nv + b) * nu + a, acc * scale);
}

// Projector for the separable geometry (detector columns horizontal, rows
// vertical).  All rays of one detector column share their major axis, their
// ray parameter tau at every plane and their in-plane (x or y) sample
// position; only the z coordinate depends on the row.  Each wave therefore
// first tabulates, for its column, one entry per plane in LDS (the planes are
// spread over the 64 lanes): the voxel offset of the in-plane tap pair and its
// weight.  The sampling loop then reads the entry (a broadcast LDS read),
// steps z = s_z + tau * D_z(row), which is linear in the plane, and does the
// bilinear interpolation.
struct PlaneEntry {
    int off;   // offset of the (plane, in-plane tap, z = -2 pad) voxel in the padded copy
    float wa;  // weight of the second in-plane tap
};


// Epilogue of the separable projector, for ray (v, a, b) with value
// l = (A mu)[ray] and ray-length factor L = h|D|/|D_m|:
//   kProjPlain:    out[vl][b][a] = l;
//   kProjResidual: r = y[v][b][a] - l rounded to PT, out[vl][a][b] = r * L
//                  (the transposed, scaled copy A^T reads) and the block's
//                  sum of r^2 (FP64) in partials[block];
//   kProjEmtr:     OS-EMTR subset terms (eq. 3): out[vl][a][b] =
//                  (e^-l - e^-y) L and out2[vl][a][b] = e^-l pi[v][b][a] L;
//   kProjNorm:     only the block's sum of (y - l)^2.
// vl is the view's index in the launched subset, v = view0 + vl * step.
constexpr int kProjPlain = 0, kProjResidual = 1, kProjEmtr = 2, kProjNorm = 3;

template <typename T> __device__ __forceinline__ float round_as(float x) { return x; }
template <> __device__ __forceinline__ float round_as<_Float16>(float x) { return (float)(_Float16)x; }

// WIDE: the pair copies exceed 4 GiB, so sample addresses are formed in 64 bits.
// Waves (adjacent detector columns) per block of the separable projector:
// 4, chosen by measurement (2 was 4-7 % slower at 128^3 and 256^3 and 6 %
// slower on a 640 x 640 x 2304 FP32 grid; for BF16 copies of grids 512 or more
// wide 2 was faster until the z coordinate stepped in fixed point, after which
// 4 is faster there too, 296 -> 280 ms at 512^3).  The kernel takes the count
// from its block size.
static int proj_pw(const Level &, int) { return 4; }

template <typename VT, typename PT, int MODE, typename TB, bool WIDE>
__global__ __launch_bounds__(256) void k_project_sep(const VT *__restrict__ vtx, const VT *__restrict__ vty,
                                                     PT *__restrict__ out, PT *__restrict__ out2,
                                                     const TB *__restrict__ y, const float *__restrict__ pi,
                                                     double *__restrict__ partials, const ViewIdx *__restrict__ views,
                                                     const ColD *__restrict__ cols, int nx, int ny, int nz, int nu,
                                                     int nv, double h, int view0, int view_step, int tab_len) {
    extern __shared__ PlaneEntry tab[];
    const int lane = threadIdx.x & 63;
    // wave index made scalar: the column descriptor, the copy's base and the
    // table's address then live in scalar registers
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int pw = blockDim.x >> 6;  // waves per block: 2 or 4
    const int a = blockIdx.x * pw + w;
    const int b = blockIdx.y * 64 + lane;
    const int v = view0 + blockIdx.z * view_step;
    PlaneEntry *T = tab + w * tab_len;
    const int ac = min(a, nu - 1);  // waves past the last column build a table nobody reads
    const ColD C = cols[(long)v * nu + ac];
    const ViewIdx &V = views[v];
    const int m = C.axis;
    const double Dm = (m == 0) ? C.dx : C.dy, Da = (m == 0) ? C.dy : C.dx, rDm = (m == 0) ? C.rdx : C.rdy;
    const double sm = V.s[m], sa = V.s[1 - m];
    const int n_m = (m == 0) ? nx : ny, n_a = (m == 0) ? ny : nx;
    // pair copy of this major axis: [plane][a][z] pairs along a
    const VT *vt = (m == 0) ? vtx : vty;
    const int PA = n_a + 2 * kVolPad, PZ = nz + 2 * kVolPad;
    const int Sm = PA * PZ, Sa = PZ;
    // planes between source and detector whose in-plane sample can touch the grid
    double lo = fmax(0.0, ceil(fmin(sm, sm + Dm)));
    double hi = fmin((double)(n_m - 1), floor(fmax(sm, sm + Dm)));
    const double Ba = Da * rDm;
    clip_range(lo, hi, sa - sm * Ba, Ba, -1.5, n_a + 0.5);
    if (!(fabs(Dm) > 0.0) || !isfinite(Ba)) hi = lo - 1.0;
    const int l0 = (int)fmax(lo, 0.0), l1 = (int)fmin(hi, (double)(n_m - 1));
    for (int base = l0; base <= l1; base += 64) {
        const int l = base + lane;
        if (l <= l1) {
            const double tau = ((double)l - sm) * rDm;
            const double fa = fma(tau, Da, sa) + kVolPad;
            const double ga = floor(fa);
            PlaneEntry e;
            e.off = (l + kVolPad) * Sm + (int)ga * Sa;  // in pairs
            e.wa = (float)(fa - ga);
            T[l] = e;
        }
    }
    __syncthreads();
    const bool valid = a < nu && b < nv;
    double r2 = 0.0;
    if (valid) {
        double D[3];
        const double len = ray_setup(V, nu, nv, a, b, D);
        const double Dz = D[2];
        // planes whose z sample lies within the padded grid, for this row
        const double Bz = Dz * rDm;
        double zlo = (double)l0, zhi = (double)l1;
        clip_range(zlo, zhi, V.s[2] - sm * Bz, Bz, -1.5, nz + 0.5);
        const float scale = (float)(h * len / fabs(D[m]));
        const double szp = V.s[2] + kVolPad;
        float acc = 0.f;
        if (zlo <= zhi && isfinite(Bz)) {
            const int lz0 = (int)zlo, lz1 = (int)zhi;
            // The sample's padded z on plane l is linear in l (slope Bz), so it
            // steps from plane lz0 in 32.32 fixed point: integer part zi (the
            // lower z tap) and fraction zf (its weight), an integer add with
            // carry per plane instead of FP64 arithmetic, which issues at half
            // the FP32 rate here.  Start and slope are rounded once from FP64;
            // the drift stays below 2^-33 per plane.  The clipped range keeps
            // every sample at least half a voxel inside the padded copy.
            const double z0 = fma(((double)lz0 - sm) * rDm, Dz, szp);
            const double g0 = floor(z0), gb = floor(Bz);
            int zi = (int)g0;
            uint32_t zf = frac_u32(z0 - g0);
            const int bi = (int)gb;
            const uint32_t bf = frac_u32(Bz - gb);
#pragma unroll 2
            for (int l = lz0; l <= lz1; ++l) {
                const PlaneEntry e = T[l];
                const float wz = (float)zf * 0x1p-32f;
                // taps (a0,z0) (a1,z0) (a0,z1) (a1,z1)
                const float4 r = WIDE ? load_quad(vt + 2L * ((long)e.off + (long)zi), 0u)
                                      : load_quad(vt, 2u * (uint32_t)(e.off + zi));
                const float q0 = fmaf(wz, r.z - r.x, r.x), q1 = fmaf(wz, r.w - r.y, r.y);
                acc += fmaf(e.wa, q1 - q0, q0);
                const uint32_t nf = zf + bf;
                zi += bi + (nf < zf ? 1 : 0);
                zf = nf;
            }
        }
        const float l = acc * scale;
        if (MODE == kProjPlain) {
            store_f(out, ((long)blockIdx.z * nv + b) * nu + a, l);
        } else {
            const long gi = ((long)v * nv + b) * nu + a;           // this ray in the full stack
            const long ot = ((long)blockIdx.z * nu + a) * nv + b;  // transposed output
            const float yv = load_f(y, gi);
            if (MODE == kProjEmtr) {
                const float e = expf(-l);
                store_f(out, ot, (e - expf(-yv)) * scale);
                store_f(out2, ot, (e * pi[gi]) * scale);
            } else {
                const float r = round_as<PT>(yv - l);
                if (MODE == kProjResidual) store_f(out, ot, r * scale);
                r2 = (double)r * (double)r;
            }
        }
    }
    if (MODE == kProjResidual || MODE == kProjNorm) {
        // fixed-order block sum of r^2: within each wave, then over the waves
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) r2 += __shfl_xor(r2, o, 64);
        __shared__ double wsum[4];
        if (lane == 0) wsum[w] = r2;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int q = 0; q < pw; ++q) t += wsum[q];
            partials[((long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = t;
        }
    }
}

hipError_t launch_project_sep(const void *vtx, const void *vty, int vt_dtype, void *proj, int proj_dtype,
                              const Level &L, int view0, int view_step, int nviews_sub, hipStream_t s) {
    return launch_project_sep_mode(vtx, vty, vt_dtype, kProjPlain, proj, nullptr, proj_dtype, nullptr, MGCT_F32,
                                   nullptr, nullptr, L, view0, view_step, nviews_sub, s);
}

size_t project_sep_blocks(const Level &L, int nviews_sub, int vt_dtype) {
    const int pw = proj_pw(L, vt_dtype);
    return (size_t)((L.nu + pw - 1) / pw) * ((L.nv + 63) / 64) * nviews_sub;
}

hipError_t launch_project_sep_mode(const void *vtx, const void *vty, int vt_dtype, int mode, void *out, void *out2,
                                   int out_dtype, const void *y, int y_dtype, const float *pi, double *partials,
                                   const Level &L, int view0, int view_step, int nviews_sub, hipStream_t s) {
    const int pw = proj_pw(L, vt_dtype);
    dim3 grid((L.nu + pw - 1) / pw, (L.nv + 63) / 64, nviews_sub);
    const int tab_len = std::max(L.nx, L.ny);
    const size_t lds = pw * (size_t)tab_len * sizeof(PlaneEntry);
    const size_t copy_bytes = pair_copy_elems(L) * (vt_dtype == MGCT_F32 ? 4 : 2);
    const bool wide = copy_bytes > 0xFFFFFFF0ull;
    if (wide && mode == kProjEmtr) return hipErrorNotSupported;  // coarse grids only
#define MGCT_PROJS_W(VT, PT, MODE, TB, W)                                                                        \
    k_project_sep<VT, PT, MODE, TB, W><<<grid, 64 * pw, lds, s>>>((const VT *)vtx, (const VT *)vty, (PT *)out,         \
                                                              (PT *)out2, (const TB *)y, pi, partials, L.d_views,    \
                                                              L.d_cols, L.nx, L.ny, L.nz, L.nu, L.nv, L.h, view0,    \
                                                              view_step, tab_len)
#define MGCT_PROJS(VT, PT, MODE, TB)                                                                             \
    do {                                                                                                        \
        if (wide && MODE != kProjEmtr) MGCT_PROJS_W(VT, PT, MODE, TB, (MODE != kProjEmtr));                     \
        else MGCT_PROJS_W(VT, PT, MODE, TB, false);                                                             \
    } while (0)
#define MGCT_PROJ_VT(PT, MODE, TB)                                                                               \
    do {                                                                                                        \
        if (vt_dtype == MGCT_F32) MGCT_PROJS(float, PT, MODE, TB);                                              \
        else if (vt_dtype == MGCT_BF16) MGCT_PROJS(uint16_t, PT, MODE, TB);                                     \
        else return hipErrorInvalidValue;                                                                       \
    } while (0)
    const bool of32 = out_dtype == MGCT_F32, of16 = out_dtype == MGCT_F16;
    const bool yf32 = y_dtype == MGCT_F32, yf16 = y_dtype == MGCT_F16;
    if (mode == kProjPlain) {
        if (of32) MGCT_PROJ_VT(float, kProjPlain, float);
        else if (of16) MGCT_PROJ_VT(_Float16, kProjPlain, float);
        else return hipErrorInvalidValue;
    } else if (mode == kProjResidual) {
        if (of32 && yf32) MGCT_PROJ_VT(float, kProjResidual, float);
        else if (of32 && yf16) MGCT_PROJ_VT(float, kProjResidual, _Float16);
        else if (of16 && yf32) MGCT_PROJ_VT(_Float16, kProjResidual, float);
        else if (of16 && yf16) MGCT_PROJ_VT(_Float16, kProjResidual, _Float16);
        else return hipErrorInvalidValue;
    } else if (mode == kProjEmtr) {
        if (of32 && yf32) MGCT_PROJ_VT(float, kProjEmtr, float);
        else return hipErrorInvalidValue;
    } else if (mode == kProjNorm) {
        if (yf32) MGCT_PROJ_VT(float, kProjNorm, float);
        else if (yf16) MGCT_PROJ_VT(float, kProjNorm, _Float16);
        else return hipErrorInvalidValue;
    } else {
        return hipErrorInvalidValue;
    }
#undef MGCT_PROJ_VT
#undef MGCT_PROJS
#undef MGCT_PROJS_W
    return hipGetLastError();
}

#ifndef MGCT_PROJ_LDS
#define MGCT_PROJ_LDS 1
#endif
#ifndef MGCT_PROJ_LDS_MIN_VOX
#define MGCT_PROJ_LDS_MIN_VOX (256u * 256u * 256u)
#endif
#ifndef MGCT_PROJ_LDS_WAVES
#define MGCT_PROJ_LDS_WAVES 6
#endif

// zp += zs on 64-bit fixed-point z positions, as one VALU instruction: written
// out so that the compiler keeps one induction variable (left to itself it
// splits the low word into a second one and adds a compare per step).
__device__ __forceinline__ void z_advance(uint64_t &zp, uint64_t zs) {
    asm("v_lshl_add_u64 %0, %1, 0, %2" : "=v"(zp) : "v"(zp), "v"(zs));
}

// ------------------------------------------ LDS-staged separable projector --
//
// The Joseph sums of k_project_sep with the four bilinear taps of every sample
// served from LDS.  A block takes kLdsTC adjacent detector columns of one view
// (one wave per column, lanes = 64 consecutive rows) and reads the volume from
// the plain padded z-fastest copy vt[x][y][z] (half the bytes of the two pair
// copies).  The planes of the rays' major axis are walked in chunks of kLdsP:
// for each chunk the block stages in LDS, per plane, the in-plane rows
// [a_lo(l), a_lo(l) + n_a(l)) (a_lo from the block's own columns' taps) times
// the z values [z_lo, z_lo + n_z) (from the tile's corner rays, which bound
// every ray of the tile because z is bilinear in the ray parameter and the
// row's z slope), one coalesced run of z values per row, and every sample
// reads its taps as two pairs of adjacent LDS words.  Each staged value serves
// about 1.8 rays x 4 taps at the workloads' sampling density, where the pair
// copies delivered 16 bytes from the vector cache per sample.  A chunk whose
// window exceeds the buffer, and every chunk of a block whose columns mix x-
// and y-major rays, reads its taps from the copy directly (two 8-byte loads per
// sample).
//
// Per sample the arithmetic is k_project_sep's: the same FP64 in-plane position
// and weight, the same 32.32 fixed-point z stepping from the same FP64 start,
// the same FP32 blend in the same order, planes in increasing order; the two
// kernels return bit-identical sums.
//
// Blocks are ordered for the caches: `order` lists (view, row tile) pairs,
// views grouped by source height (views at one height sample the same z band
// in a row tile) and by angle within a group, and a pair's column tiles are
// consecutive blocks.  The blocks resident at one time then cover a few views
// of one height and row tile: one z band of the volume, which stays in the
// last-level cache while the group's views pass over it.  (Handing each XCD
// every 8th pair instead, to keep a pair's neighbouring tiles in one L2, was
// 8 % slower at 512^3; views in their natural order 13 % slower.)
constexpr int kLdsTC = 8;    // columns (waves) per block
constexpr int kLdsP = 8;     // planes per chunk (one staging buffer)
constexpr int kLdsTB = 64;   // planes per table block (one per lane)
constexpr int kLdsNQ = kLdsTB / kLdsP;  // chunks per table block
constexpr int kLdsAW = 11;   // in-plane rows per staged plane
constexpr int kLdsZW = 64;   // z values per staged row
constexpr int kLdsRows = kLdsP * kLdsAW;
constexpr int kNoTap = -0x7fffffff - 1;  // no tap of this column on the plane
static_assert(kLdsTB % kLdsP == 0 && kLdsNQ <= 64, "LDS projector tiling");

// Staging of one chunk: issue the loads (into registers), then commit them to
// an LDS buffer; the next chunk's loads are in flight while the current one is
// sampled.  Wave w stages plane w of the chunk: its in-plane rows
// ia = 4 u + lane / 16 (u < kLdsIter), z values 4 (lane mod 16) .. + 3, so the
// plane's window (a_lo, n_a) is wave-uniform.
constexpr int kLdsIter = (kLdsAW + 3) / 4;
static_assert(kLdsP == kLdsTC, "one staged plane per wave");

struct LdsStage {
    float4 val[kLdsIter];
    unsigned ok;  // bit u: rows 4u .. 4u + 3 hold this lane's row
};

// pl: the plane (absolute), alo / na: its window (wave-uniform), zl / zn: the
// chunk's z window
template <typename VT, bool WIDE>
__device__ __forceinline__ void lds_stage_issue(LdsStage &st, const VT *__restrict__ vt, int lane, bool plane_ok,
                                                int pl, int alo, int na, int zl, int zn, long Sm, long Sa) {
    const int sub = lane >> 4, zq = (lane & 15) * 4;
    const bool zok = plane_ok && zq < zn;
    const long base = (long)(pl + kVolPad) * Sm + (long)(alo + sub) * Sa + zl + zq;
    st.ok = 0u;
#pragma unroll
    for (int u = 0; u < kLdsIter; ++u) {
        const bool ok = zok && 4 * u + sub < na;
        if (WIDE) {
            st.val[u] = load_quad(vt + (ok ? base + 4 * u * Sa : 0), 0u);
        } else {
            st.val[u] = load_quad(vt, ok ? (uint32_t)(base + 4 * u * Sa) : 0u);
        }
        st.ok |= ok ? (1u << u) : 0u;
    }
}

// buf: the LDS array (passed as such so that the accesses stay LDS accesses),
// base: the plane's first element in the buffer
__device__ __forceinline__ void lds_stage_commit(const LdsStage &st, int lane, float (&buf)[2 * kLdsRows * kLdsZW],
                                                 int base) {
    const int o = base + (lane >> 4) * kLdsZW + (lane & 15) * 4;
#pragma unroll
    for (int u = 0; u < kLdsIter; ++u)
        if (st.ok & (1u << u)) *reinterpret_cast<float4 *>(&buf[o + 4 * u * kLdsZW]) = st.val[u];
}

template <typename VT, typename PT, int MODE, typename TB, bool WIDE>
__global__ __launch_bounds__(64 * kLdsTC, MGCT_PROJ_LDS_WAVES) void k_project_lds(const VT *__restrict__ vt, PT *__restrict__ out,
                                                             const TB *__restrict__ y, double *__restrict__ partials,
                                                             const ViewIdx *__restrict__ views,
                                                             const ColD *__restrict__ cols, const int *__restrict__ order,
                                                             int n_ct, int n_t, int n_rt, int nx, int ny, int nz,
                                                             int nu, int nv, double h) {
    __shared__ float S[2 * kLdsRows * kLdsZW];  // two staging buffers
    __shared__ int AI[kLdsTC][kLdsTB];
    __shared__ int WL[kLdsTB], NA[kLdsTB];
    __shared__ int CZ[kLdsNQ], CN[kLdsNQ], CD[kLdsNQ];
    __shared__ int s_l0, s_l1, s_and, s_or;
    __shared__ double wsum[kLdsTC];

    const unsigned bid = blockIdx.x;
    const int ct = (int)(bid % (unsigned)n_ct);
    const int t = (int)(bid / (unsigned)n_ct);
    if (t >= n_t) return;  // whole block, before any barrier
    const int e = order[t];
    const int v = e / n_rt, rt = e - (e / n_rt) * n_rt;

    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int a = ct * kLdsTC + w;
    const int b = rt * 64 + lane;
    const bool colok = a < nu;
    const int ac = min(a, nu - 1);
    const ColD C = cols[(long)v * nu + ac];
    const ViewIdx &V = views[v];
    const int m = C.axis;
    const double Dm = (m == 0) ? C.dx : C.dy, Da = (m == 0) ? C.dy : C.dx, rDm = (m == 0) ? C.rdx : C.rdy;
    const double sm = V.s[m], sa = V.s[1 - m];
    const int n_m = (m == 0) ? nx : ny, n_a = (m == 0) ? ny : nx;
    const int PY = ny + 2 * kVolPad, PZ = nz + 2 * kVolPad;
    // copy strides of this column's plane and in-plane axes (vt is [x][y][z])
    const long Sm = (m == 0) ? (long)PY * PZ : (long)PZ;
    const long Sa = (m == 0) ? (long)PZ : (long)PY * PZ;
    double lo = fmax(0.0, ceil(fmin(sm, sm + Dm)));
    double hi = fmin((double)(n_m - 1), floor(fmax(sm, sm + Dm)));
    const double Ba = Da * rDm;
    clip_range(lo, hi, sa - sm * Ba, Ba, -1.5, n_a + 0.5);
    if (!(fabs(Dm) > 0.0) || !isfinite(Ba) || !colok) hi = lo - 1.0;
    const int l0 = (int)fmax(lo, 0.0), l1 = (int)fmin(hi, (double)(n_m - 1));

    if (threadIdx.x == 0) {
        s_l0 = 0x7fffffff;
        s_l1 = -1;
        s_and = 3;
        s_or = 0;
    }
    __syncthreads();
    if (lane == 0 && colok) {
        if (l0 <= l1) {
            atomicMin(&s_l0, l0);
            atomicMax(&s_l1, l1);
        }
        atomicAnd(&s_and, 1 << m);
        atomicOr(&s_or, 1 << m);
    }
    __syncthreads();
    // block-uniform values read from LDS, made scalar
    const int L0 = __builtin_amdgcn_readfirstlane(s_l0), L1 = __builtin_amdgcn_readfirstlane(s_l1);
    const bool mixed = __builtin_amdgcn_readfirstlane(s_and) != __builtin_amdgcn_readfirstlane(s_or);

    // this lane's ray
    const bool valid = colok && b < nv;
    double D[3];
    const double len = ray_setup(V, nu, nv, ac, min(b, nv - 1), D);
    const double Dz = D[2];
    const double Bz = Dz * rDm;
    double zlo = (double)l0, zhi = (double)l1;
    clip_range(zlo, zhi, V.s[2] - sm * Bz, Bz, -1.5, nz + 0.5);
    const bool act = valid && zlo <= zhi && isfinite(Bz);
    const int lz0 = act ? (int)zlo : 0x7fffffff, lz1 = act ? (int)zhi : -1;
    const float scale = (float)(h * len / fabs(D[m]));
    const double szp = V.s[2] + kVolPad;
    // z position in 32.32 fixed point (integer part in the high word: the
    // copy's z index; fraction in the low word) and its step per plane, as
    // one 64-bit addition (a carry into the high word is the index step)
    uint64_t zp = 0, zs = 0;
    if (act) {
        const double z0 = fma(((double)lz0 - sm) * rDm, Dz, szp);
        const double g0 = floor(z0), gb = floor(Bz);
        zp = ((uint64_t)(uint32_t)(int)g0 << 32) | frac_u32(z0 - g0);
        zs = ((uint64_t)(uint32_t)(int)gb << 32) | frac_u32(Bz - gb);
    }
    auto zi = [&]() { return (int)(uint32_t)(zp >> 32); };
    auto zf = [&]() { return (uint32_t)zp; };
    // planes on which every active lane of this wave samples: no per-sample test there
    int f_lo = act ? lz0 : -0x7fffffff, f_hi = act ? lz1 : 0x7fffffff;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        f_lo = max(f_lo, __shfl_xor(f_lo, o, 64));
        f_hi = min(f_hi, __shfl_xor(f_hi, o, 64));
    }
    f_lo = __builtin_amdgcn_readfirstlane(f_lo);
    f_hi = __builtin_amdgcn_readfirstlane(f_hi);
    float acc = 0.f;

    for (int tb = L0; tb <= L1; tb += kLdsTB) {
        // A: this column's tap and weight on plane tb + lane
        int my_ai = kNoTap;
        float my_wa = 0.f;
        {
            const int l = tb + lane;
            if (l >= l0 && l <= l1) {
                const double tau = ((double)l - sm) * rDm;
                const double fa = fma(tau, Da, sa) + kVolPad;
                const double ga = floor(fa);
                my_ai = (int)ga;
                my_wa = (float)(fa - ga);
            }
            AI[w][lane] = my_ai;
        }
        __syncthreads();
        // B (wave 0): per-plane in-plane windows (lane = plane), per-chunk z
        // windows from the tile's corner rays (lane = chunk), and whether each
        // chunk fits the buffers
        if (w == 0) {
            int alo = 0x7fffffff, ahi = kNoTap;
#pragma unroll
            for (int c = 0; c < kLdsTC; ++c) {
                const int ai = AI[c][lane];
                if (ai != kNoTap) {
                    alo = min(alo, ai);
                    ahi = max(ahi, ai);
                }
            }
            const int na = ahi >= alo ? ahi - alo + 2 : 0;
            WL[lane] = alo;
            NA[lane] = na;
            const unsigned long long over = __ballot(na > kLdsAW);
            if (lane < kLdsNQ) {
                const int cs = tb + lane * kLdsP, ce = min(cs + kLdsP - 1, L1);
                int zl = 0, zn = 0;
                if (cs <= L1 && !mixed) {
                    const int c0 = ct * kLdsTC, c1 = min(c0 + kLdsTC - 1, nu - 1);
                    const int b0 = rt * 64, b1 = min(b0 + 63, nv - 1);
                    double zmin = HUGE_VAL, zmax = -HUGE_VAL;
                    for (int q = 0; q < 4; ++q) {
                        const int cc = (q & 1) ? c1 : c0, bb = (q & 2) ? b1 : b0;
                        const ColD Cq = cols[(long)v * nu + cc];
                        const double rq = (m == 0) ? Cq.rdx : Cq.rdy;
                        const double dzq = (V.d[2] + (cc - 0.5 * (nu - 1)) * V.u[2] + (bb - 0.5 * (nv - 1)) * V.v[2]) -
                                           V.s[2];
                        for (int r = 0; r < 2; ++r) {
                            const double z = fma(((double)(r ? ce : cs) - sm) * rq, dzq, szp);
                            zmin = fmin(zmin, z);
                            zmax = fmax(zmax, z);
                        }
                    }
                    const double flo = fmax(floor(zmin) - 1.0, 0.0), fhi = fmin(floor(zmax) + 2.0, (double)(PZ - 1));
                    if (isfinite(flo) && isfinite(fhi) && fhi >= flo && fhi - flo + 1.0 <= (double)kLdsZW) {
                        zl = (int)flo;
                        zn = (int)(fhi - flo) + 1;
                    } else {
                        zn = kLdsZW + 1;  // does not fit
                    }
                }
                CZ[lane] = zl;
                CN[lane] = zn;
                const unsigned grp = (unsigned)((over >> (lane * kLdsP)) & ((1ull << kLdsP) - 1));
                CD[lane] = (mixed || zn > kLdsZW || grp != 0u) ? 1 : 0;
            }
        }
        __syncthreads();
        // this lane's plane's offset in a staging buffer, relative to z = 0
        const int my_off =
            my_ai == kNoTap ? 0 : ((lane & (kLdsP - 1)) * kLdsAW + (my_ai - WL[lane])) * kLdsZW - CZ[lane / kLdsP];
        const int tend = min(tb + kLdsTB - 1, L1);
        const int nq = (tend - tb) / kLdsP + 1;
        // C: chunks, staging double-buffered; a chunk whose window does not
        // fit is sampled from the copy directly
        LdsStage st;
        // the window of plane w of chunk q (wave-uniform)
        auto issue = [&](int q) {
            const int cs = tb + q * kLdsP, pl = cs + w, j = q * kLdsP + w;
            lds_stage_issue<VT, WIDE>(st, vt, lane, pl <= L1, pl, __builtin_amdgcn_readfirstlane(WL[j]),
                                      __builtin_amdgcn_readfirstlane(NA[j]), __builtin_amdgcn_readfirstlane(CZ[q]),
                                      __builtin_amdgcn_readfirstlane(CN[q]), Sm, Sa);
        };
        const int wplane = w * kLdsAW * kLdsZW;  // this wave's plane in a buffer
        bool dnext = __builtin_amdgcn_readfirstlane(CD[0]) != 0;
        if (!dnext) {
            issue(0);
            lds_stage_commit(st, lane, S, wplane);
        }
        __syncthreads();
        for (int q = 0; q < nq; ++q) {
            const int cs = tb + q * kLdsP, ce = min(cs + kLdsP - 1, L1);
            const bool direct = dnext;
            if (q + 1 < nq) {
                dnext = __builtin_amdgcn_readfirstlane(CD[q + 1]) != 0;
                if (!dnext) issue(q + 1);
            }
            if (act) {
                const int sb = (q & 1) * kLdsRows * kLdsZW;
                // one sample on plane l (wave-uniform): taps from LDS or, for a
                // direct chunk, from the copy
                auto lds_sample = [&](int l) {
                    const int j = l - tb;
                    const float wa = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(my_wa), j));
                    const int o = sb + __builtin_amdgcn_readlane(my_off, j) + zi();
                    const float x00 = S[o], x01 = S[o + 1], x10 = S[o + kLdsZW], x11 = S[o + kLdsZW + 1];
                    const float wz = (float)zf() * 0x1p-32f;
                    const float q0 = fmaf(wz, x01 - x00, x00), q1 = fmaf(wz, x11 - x10, x10);
                    acc += fmaf(wa, q1 - q0, q0);
                    z_advance(zp, zs);
                };
                auto direct_sample = [&](int l) {
                    const int j = l - tb;
                    const float wa = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(my_wa), j));
                    const int ai = __builtin_amdgcn_readlane(my_ai, j);
                    const long g = (long)(l + kVolPad) * Sm + (long)ai * Sa + zi();
                    float2 p0, p1;
                    if (WIDE) {
                        p0 = load_pair(vt + g, 0u);
                        p1 = load_pair(vt + g + Sa, 0u);
                    } else {
                        p0 = load_pair(vt, (uint32_t)g);
                        p1 = load_pair(vt, (uint32_t)(g + Sa));
                    }
                    const float wz = (float)zf() * 0x1p-32f;
                    const float q0 = fmaf(wz, p0.y - p0.x, p0.x), q1 = fmaf(wz, p1.y - p1.x, p1.x);
                    acc += fmaf(wa, q1 - q0, q0);
                    z_advance(zp, zs);
                };
                // planes where every active lane samples need no per-lane test
                const int f0 = max(cs, f_lo), f1 = min(ce, f_hi);
                auto run = [&](auto smp) {
                    if (f0 > f1) {
                        for (int l = cs; l <= ce; ++l)
                            if (l >= lz0 && l <= lz1) smp(l);
                        return;
                    }
                    for (int l = cs; l < f0; ++l)
                        if (l >= lz0) smp(l);
                    int l = f0;
                    for (; l + 3 <= f1; l += 4) {
                        smp(l);
                        smp(l + 1);
                        smp(l + 2);
                        smp(l + 3);
                    }
                    for (; l <= f1; ++l) smp(l);
                    for (l = f1 + 1; l <= ce; ++l)
                        if (l <= lz1) smp(l);
                };
                if (direct) {
                    for (int l = cs; l <= ce; ++l)
                        if (l >= lz0 && l <= lz1) direct_sample(l);
                } else if (f0 > f1) {
                    run(lds_sample);
                } else {
                    for (int l = cs; l < f0; ++l)
                        if (l >= lz0) lds_sample(l);
                    // every active lane samples planes f0..f1: the taps of the
                    // next plane are read while this plane is blended (two
                    // register sets in turn; past f1 the last address is read
                    // again and the values are not used)
                    int o = sb + __builtin_amdgcn_readlane(my_off, f0 - tb) + zi();
                    float a00 = S[o], a01 = S[o + 1], a10 = S[o + kLdsZW], a11 = S[o + kLdsZW + 1];
                    float b00, b01, b10, b11;
                    auto blend = [&](int l, float x00, float x01, float x10, float x11, float wz) {
                        const float wa = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(my_wa), l - tb));
                        const float q0 = fmaf(wz, x01 - x00, x00), q1 = fmaf(wz, x11 - x10, x10);
                        acc += fmaf(wa, q1 - q0, q0);
                    };
                    auto step = [&]() {
                        const float wz = (float)zf() * 0x1p-32f;
                        z_advance(zp, zs);
                        return wz;
                    };
                    // two samples per trip (the a-set is carried to the next
                    // trip, the b-set is used within it); one sample left over
                    int l = f0;
                    for (; l + 1 <= f1; l += 2) {
                        float wz = step();
                        o = sb + __builtin_amdgcn_readlane(my_off, l + 1 - tb) + zi();
                        b00 = S[o];
                        b01 = S[o + 1];
                        b10 = S[o + kLdsZW];
                        b11 = S[o + kLdsZW + 1];
                        blend(l, a00, a01, a10, a11, wz);
                        wz = step();
                        const int on = sb + __builtin_amdgcn_readlane(my_off, min(l + 2, f1) - tb) + zi();
                        o = l + 2 <= f1 ? on : o;
                        a00 = S[o];
                        a01 = S[o + 1];
                        a10 = S[o + kLdsZW];
                        a11 = S[o + kLdsZW + 1];
                        blend(l + 1, b00, b01, b10, b11, wz);
                    }
                    if (l == f1) blend(l, a00, a01, a10, a11, step());
                    for (int l = f1 + 1; l <= ce; ++l)
                        if (l <= lz1) lds_sample(l);
                }
            }
            if (q + 1 < nq && !dnext) lds_stage_commit(st, lane, S, ((q + 1) & 1) * kLdsRows * kLdsZW + wplane);
            __syncthreads();
        }
    }

    double r2 = 0.0;
    if (valid) {
        const float lv = acc * scale;
        if (MODE == kProjPlain) {
            store_f(out, ((long)v * nv + b) * nu + a, lv);
        } else {
            const long gi = ((long)v * nv + b) * nu + a;
            const long ot = ((long)v * nu + a) * nv + b;
            const float yv = load_f(y, gi);
            const float r = round_as<PT>(yv - lv);
            if (MODE == kProjResidual) store_f(out, ot, r * scale);
            r2 = (double)r * (double)r;
        }
    }
    if (MODE == kProjResidual || MODE == kProjNorm) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) r2 += __shfl_xor(r2, o, 64);
        if (lane == 0) wsum[w] = r2;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int q = 0; q < kLdsTC; ++q) s += wsum[q];
            partials[(long)t * n_ct + ct] = s;
        }
    }
}

bool project_lds_ok(const Level &L, int nviews_sub, int variant) {
    if (!L.separable || !L.d_order || nviews_sub != L.nviews || variant == MGCT_PROJECTOR_GATHER) return false;
    if (variant == MGCT_PROJECTOR_STAGED) return true;
    // automatic: the staged projector where the volume outgrows the caches
    return MGCT_PROJ_LDS && (size_t)L.nx * L.ny * L.nz >= (size_t)MGCT_PROJ_LDS_MIN_VOX;
}

size_t project_lds_blocks(const Level &L) {
    const int n_ct = (L.nu + kLdsTC - 1) / kLdsTC;
    return (size_t)n_ct * L.n_rt * L.nviews;
}

size_t project_lds_blocks_judge(const Level &L) {
    const int n_ct = (L.nu + kLdsTC - 1) / kLdsTC;
    return (size_t)n_ct * L.n_t_judge;
}

size_t plain_copy_elems(const Level &L) { return L.padded_vox(); }

hipError_t launch_project_lds_mode(const void *vt, int vt_dtype, int mode, void *out, int out_dtype, const void *y,
                                   int y_dtype, double *partials, const Level &L, hipStream_t s, const int *order,
                                   int n_t) {
    const int n_ct = (L.nu + kLdsTC - 1) / kLdsTC;
    if (!order) {
        order = L.d_order;
        n_t = L.n_rt * L.nviews;
    }
    if (!order || n_t <= 0) return hipErrorInvalidValue;
    const unsigned nblk = (unsigned)n_ct * (unsigned)n_t;
    const size_t copy_bytes = L.padded_vox() * (vt_dtype == MGCT_F32 ? 4 : 2);
    const bool wide = copy_bytes > 0xFFFFFFF0ull;
#define MGCT_LDS_W(VT, PT, MODE, TB, W)                                                                           \
    k_project_lds<VT, PT, MODE, TB, W><<<nblk, 64 * kLdsTC, 0, s>>>(                                             \
        (const VT *)vt, (PT *)out, (const TB *)y, partials, L.d_views, L.d_cols, order, n_ct, n_t, L.n_rt, L.nx,     \
        L.ny, L.nz, L.nu, L.nv, L.h)
#define MGCT_LDS(VT, PT, MODE, TB)                                \
    do {                                                          \
        if (wide) MGCT_LDS_W(VT, PT, MODE, TB, true);             \
        else MGCT_LDS_W(VT, PT, MODE, TB, false);                 \
    } while (0)
#define MGCT_LDS_VT(PT, MODE, TB)                                                                                 \
    do {                                                                                                        \
        if (vt_dtype == MGCT_F32) MGCT_LDS(float, PT, MODE, TB);                                                \
        else if (vt_dtype == MGCT_BF16) MGCT_LDS(uint16_t, PT, MODE, TB);                                       \
        else return hipErrorInvalidValue;                                                                       \
    } while (0)
    const bool of32 = out_dtype == MGCT_F32, of16 = out_dtype == MGCT_F16;
    const bool yf32 = y_dtype == MGCT_F32, yf16 = y_dtype == MGCT_F16;
    if (mode == kProjPlain) {
        if (of32) MGCT_LDS_VT(float, kProjPlain, float);
        else if (of16) MGCT_LDS_VT(_Float16, kProjPlain, float);
        else return hipErrorInvalidValue;
    } else if (mode == kProjResidual) {
        if (of32 && yf32) MGCT_LDS_VT(float, kProjResidual, float);
        else if (of32 && yf16) MGCT_LDS_VT(float, kProjResidual, _Float16);
        else if (of16 && yf32) MGCT_LDS_VT(_Float16, kProjResidual, float);
        else if (of16 && yf16) MGCT_LDS_VT(_Float16, kProjResidual, _Float16);
        else return hipErrorInvalidValue;
    } else if (mode == kProjNorm) {
        if (yf32) MGCT_LDS_VT(float, kProjNorm, float);
        else if (yf16) MGCT_LDS_VT(float, kProjNorm, _Float16);
        else return hipErrorInvalidValue;
    } else {
        return hipErrorInvalidValue;
    }
#undef MGCT_LDS_VT
#undef MGCT_LDS
#undef MGCT_LDS_W
    return hipGetLastError();
}

hipError_t launch_project(const void *vt, int vt_dtype, void *proj, int proj_dtype, const Level &L, int view0,
                          int view_step, int nviews_sub, hipStream_t s) {
    dim3 grid((L.nu + 3) / 4, (L.nv + 63) / 64, nviews_sub);
    const long avs = L.separable ? (long)L.nu : (long)L.nu * L.nv;
    const long ars = L.axis_row_stride;
#define MGCT_PROJ(VT, PT)                                                                                       \
    k_project<VT, PT><<<grid, 256, 0, s>>>((const VT *)vt, (PT *)proj, L.d_views, L.d_axis, avs, ars, L.nx, L.ny, \
                                           L.nz, L.nu, L.nv, L.h, view0, view_step)
    if (vt_dtype == MGCT_F32 && proj_dtype == MGCT_F32) MGCT_PROJ(float, float);
    else if (vt_dtype == MGCT_F32 && proj_dtype == MGCT_F16) MGCT_PROJ(float, _Float16);
    else if (vt_dtype == MGCT_BF16 && proj_dtype == MGCT_F32) MGCT_PROJ(uint16_t, float);
    else if (vt_dtype == MGCT_BF16 && proj_dtype == MGCT_F16) MGCT_PROJ(uint16_t, _Float16);
    else return hipErrorInvalidValue;
#undef MGCT_PROJ
    return hipGetLastError();
}

// ------------------------------------------- data pre-scale and transpose --

// pt[vl][a][b] = proj[vl][b][a] * h|D|/|D_m| of ray (view0 + vl*step, a, b).
template <typename PT, typename OT>
__global__ __launch_bounds__(256) void k_scale_transpose(const PT *__restrict__ proj, OT *__restrict__ pt,
                                                         const ViewIdx *__restrict__ views,
                                                         const uint8_t *__restrict__ axis, long axis_view_stride,
                                                         long axis_row_stride, int nu, int nv, double h, int view0,
                                                         int view_step) {
    __shared__ float tile[64][65];
    const int a0 = blockIdx.x * 64, b0 = blockIdx.y * 64, vl = blockIdx.z;
    const int v = view0 + vl * view_step;
    const ViewIdx &V = views[v];
    const int t = threadIdx.x;
#pragma unroll 4
    for (int r = 0; r < 16; ++r) {
        int bl = (t >> 6) + 4 * r, al = t & 63;
        int b = b0 + bl, a = a0 + al;
        float val = 0.f;
        if (a < nu && b < nv) {
            double D[3];
            double len = ray_setup(V, nu, nv, a, b, D);
            int m = axis[v * axis_view_stride + b * axis_row_stride + a];
            float scale = (float)(h * len / fabs(D[m]));
            val = load_f(proj, ((long)vl * nv + b) * nu + a) * scale;
        }
        tile[bl][al] = val;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        int al = (t >> 6) + 4 * r, bl = t & 63;
        int b = b0 + bl, a = a0 + al;
        if (a < nu && b < nv) store_f(pt, ((long)vl * nu + a) * nv + b, tile[bl][al]);
    }
}

hipError_t launch_scale_transpose_stack(const void *proj, int proj_dtype, void *pt, int pt_dtype, const Level &L,
                                        int view0, int view_step, int nviews_sub, hipStream_t s) {
    dim3 grid((L.nu + 63) / 64, (L.nv + 63) / 64, nviews_sub);
    const long avs = L.separable ? (long)L.nu : (long)L.nu * L.nv;
#define MGCT_ST(PT, OT)                                                                                           \
    k_scale_transpose<PT, OT><<<grid, 256, 0, s>>>((const PT *)proj, (OT *)pt, L.d_views, L.d_axis, avs,          \
                                                   L.axis_row_stride, L.nu, L.nv, L.h, view0, view_step)
    if (proj_dtype == MGCT_F32 && pt_dtype == MGCT_F32) MGCT_ST(float, float);
    else if (proj_dtype == MGCT_F16 && pt_dtype == MGCT_F32) MGCT_ST(_Float16, float);
    else if (proj_dtype == MGCT_F32 && pt_dtype == MGCT_F16) MGCT_ST(float, _Float16);
    else if (proj_dtype == MGCT_F16 && pt_dtype == MGCT_F16) MGCT_ST(_Float16, _Float16);
    else return hipErrorInvalidValue;
#undef MGCT_ST
    return hipGetLastError();
}

// OS-EMTR subset terms (eq. 3) fused with the transposition for the
// back-projector: for ray (v = view0 + vl*step, a, b) with projection l,
// data y and support projection pi, num = e^-l - e^-y and den = e^-l pi;
// pt_num[vl][a][b] = num * L and pt_den[vl][a][b] = den * L with
// L = h|D|/|D_m| (the ray-length factor of A^T).  l is [nsub][nv][nu];
// y and pi are full stacks [V][nv][nu].
__global__ __launch_bounds__(256) void k_emtr_terms_t(const float *__restrict__ l, const float *__restrict__ y,
                                                      const float *__restrict__ pi, float *__restrict__ pt_num,
                                                      float *__restrict__ pt_den, const ViewIdx *__restrict__ views,
                                                      const uint8_t *__restrict__ axis, long axis_view_stride,
                                                      long axis_row_stride, int nu, int nv, double h, int view0,
                                                      int view_step) {
    __shared__ float tn[64][65], td[64][65];
    const int a0 = blockIdx.x * 64, b0 = blockIdx.y * 64, vl = blockIdx.z;
    const int v = view0 + vl * view_step;
    const ViewIdx &V = views[v];
    const int t = threadIdx.x;
#pragma unroll 4
    for (int r = 0; r < 16; ++r) {
        const int bl = (t >> 6) + 4 * r, al = t & 63;
        const int b = b0 + bl, a = a0 + al;
        float vn = 0.f, vd = 0.f;
        if (a < nu && b < nv) {
            double D[3];
            const double len = ray_setup(V, nu, nv, a, b, D);
            const int m = axis[v * axis_view_stride + b * axis_row_stride + a];
            const float scale = (float)(h * len / fabs(D[m]));
            const long g = ((long)v * nv + b) * nu + a;
            const float e = expf(-l[((long)vl * nv + b) * nu + a]);
            vn = (e - expf(-y[g])) * scale;
            vd = (e * pi[g]) * scale;
        }
        tn[bl][al] = vn;
        td[bl][al] = vd;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int al = (t >> 6) + 4 * r, bl = t & 63;
        const int b = b0 + bl, a = a0 + al;
        if (a < nu && b < nv) {
            const long o = ((long)vl * nu + a) * nv + b;
            pt_num[o] = tn[bl][al];
            pt_den[o] = td[bl][al];
        }
    }
}

hipError_t launch_emtr_terms_t(const float *l, const float *y, const float *pi, float *pt_num, float *pt_den,
                               const Level &L, int view0, int view_step, int nviews_sub, hipStream_t s) {
    dim3 grid((L.nu + 63) / 64, (L.nv + 63) / 64, nviews_sub);
    const long avs = L.separable ? (long)L.nu : (long)L.nu * L.nv;
    k_emtr_terms_t<<<grid, 256, 0, s>>>(l, y, pi, pt_num, pt_den, L.d_views, L.d_axis, avs, L.axis_row_stride, L.nu,
                                        L.nv, L.h, view0, view_step);
    return hipGetLastError();
}

// -------------------------------------------------------- back-projector --

// W consecutive values of one detector column from element i, as one access.
template <int W> __device__ __forceinline__ void load_win(const float *p, uint32_t i, float (&v)[W]) {
    if constexpr (W == 4) {
        const float4 r = load_quad(p, i);
        v[0] = r.x, v[1] = r.y, v[2] = r.z, v[3] = r.w;
    } else {
        __builtin_memcpy(v, __builtin_assume_aligned(reinterpret_cast<const char *>(p) + i * 4u, 4), 4 * W);
    }
}
template <int W> __device__ __forceinline__ void load_win(const _Float16 *p, uint32_t i, float (&v)[W]) {
    _Float16 h[W];
    __builtin_memcpy(h, __builtin_assume_aligned(reinterpret_cast<const char *>(p) + i * 2u, 2), 2 * W);
#pragma unroll
    for (int t = 0; t < W; ++t) v[t] = (float)h[t];
}

// The hat max(0, 1 - |d|).  As 1 - |d| never exceeds 1 it equals the clamp
// of 1 - |d| to [0, 1], which the compiler folds into the subtraction's
// output clamp: one instruction instead of two (same value).
__device__ __forceinline__ float hat(float d) { return fminf(fmaxf(1.f - fabsf(d), 0.f), 1.f); }

// One detector column at a voxel plane, as the z windows of the transpose
// use it.  Detector row b sits at z = zc + tz b on the plane (voxel units);
// the voxel z = zw0 + u (u = 0, 1, ... over the wave's z values) sees the
// row at b*(u) = (zw0 + u - zc) / tz.  With R0 the row nearest b*(0), the
// window start b*(u) - |1/tz| is R0 + bq + u rtz and the hat argument of row
// R0 + dl is tz dl + C - u, C = zc + tz R0 - zw0 (|C| <= |tz| / 2).  These
// are formed in FP64 once per column; per voxel everything is FP32 (FP64
// instructions issue at half the FP32 rate here): the products tzh dl are
// exact inside the FMA, tz = tzh + tzl carries 48 bits, and the argument of
// every row that can have weight errs by about 1e-7.  The window start only
// moves a window edge, where the row it drops has a weight of order 1e-5 tz
// at most and the row it adds has weight 0.
struct WinCol {
    float R0;        // reference row (an integer, |R0| <= 2^20)
    float bq;        // window start of u = 0 relative to R0
    float C;         // z of row R0 relative to zw0
    float tzh, tzl;  // row spacing along z, split in two FP32 parts
    float rtz;       // 1 / tz (|rtz| is the half-width of the window in rows)
};

__device__ __forceinline__ WinCol win_col(double zc, double tz, double rtz, double zw0) {
    const double B = (zw0 - zc) * rtz;  // row position of z = zw0
    const double R0 = fmin(fmax(rint(B), -1048576.0), 1048576.0);
    WinCol w;
    w.R0 = (float)R0;
    w.bq = (float)((B - R0) - fabs(rtz));
    w.C = (float)fma(tz, R0, zc - zw0);
    w.tzh = (float)tz;
    w.tzl = (float)(tz - (double)w.tzh);
    w.rtz = (float)rtz;
    return w;
}

// First row of a W-row window for the voxel at u (clamped so that the window
// stays on the detector: R0 + dl in [0, nv - W]) and the hat argument of that
// row.
__device__ __forceinline__ void win_start(const WinCol &w, float u, float hi, float &dl, float &d0) {
    dl = __builtin_amdgcn_fmed3f(ceilf(fmaf(u, w.rtz, w.bq)), -w.R0, hi);
    d0 = fmaf(w.tzl, dl, fmaf(w.tzh, dl, -u) + w.C);
}

// One column's detector-row sums for the wave's KZ voxels (z = zw0 + u[q]):
// rows R0 + dl .. R0 + dl + W-1, hat weights 1 - |z_row - z|.
template <int W, int KZ, int NP, typename PT>
__device__ __forceinline__ void bp_window(const PT *col0, const PT *col1, int nv, const WinCol &w,
                                          const float (&u)[KZ], float (&s)[NP][KZ]) {
    const float hi = (float)(nv - W) - w.R0;
#pragma unroll
    for (int q = 0; q < KZ; ++q) {
        float dl, d0;
        win_start(w, u[q], hi, dl, d0);
        const int bs = (int)(dl + w.R0);
        float v0[W], v1[W];
        load_win<W>(col0, (uint32_t)bs, v0);
        if (NP > 1) load_win<W>(col1, (uint32_t)bs, v1);
        float s0 = 0.f, s1 = 0.f;
#pragma unroll
        for (int t = 0; t < W; ++t) {
            const float d = (t == 0) ? d0 : fmaf((float)t, w.tzh, d0);
            const float h = hat(d);
            s0 = fmaf(h, v0[t], s0);
            if (NP > 1) s1 = fmaf(h, v1[t], s1);
        }
        s[0][q] = s0;
        if (NP > 1) s[NP - 1][q] = s1;
    }
}

// The same sums for any row spacing: the rows within one voxel of z are
// fewer than 2 hw + 1 (hw = |1/tz|), so a fixed window of 3 (hw < 1.5) or 4
// (hw < 2) consecutive rows holds them, else a window of floor(2 hw + 1) + 1
// rows (one spare row against the rounding of hw).
template <int KZ, int NP, typename PT>
__device__ __forceinline__ void bp_column_sums(const PT *col0, const PT *col1, int nv, const WinCol &w,
                                               const float (&u)[KZ], float (&s)[NP][KZ]) {
    const float hw = fabsf(w.rtz);
    if (hw < 1.5f && nv >= 3) {
        bp_window<3, KZ, NP, PT>(col0, col1, nv, w, u, s);
    } else if (hw < 2.f && nv >= 4) {
        bp_window<4, KZ, NP, PT>(col0, col1, nv, w, u, s);
    } else {
        const int nb = min((int)(2.f * hw + 1.f) + 1, nv);
        const float hi = (float)(nv - nb) - w.R0;
#pragma unroll
        for (int q = 0; q < KZ; ++q) {
            float dl, d0;
            win_start(w, u[q], hi, dl, d0);
            const int bs = (int)(dl + w.R0);
            float s0 = 0.f, s1 = 0.f;
            for (int t = 0; t < nb; ++t) {
                const float h = hat(fmaf((float)t, w.tzh, d0));
                s0 = fmaf(h, load_f(col0, bs + t), s0);
                if (NP > 1) s1 = fmaf(h, load_f(col1, bs + t), s1);
            }
            s[0][q] = s0;
            if (NP > 1) s[NP - 1][q] = s1;
        }
    }
}

// Detector column of the ray through (px, py, .); only used to bound the
// candidate columns (with a margin), so an approximate reciprocal will do.
__device__ __forceinline__ float column_coord(const SepView &S, float px, float py) {
    return (S.an0 + S.an1 * px + S.an2 * py) * __builtin_amdgcn_rcpf(S.ad0 + S.ad1 * px + S.ad2 * py);
}

// What the column loop of bp_part needs of one column at a half-wave's
// plane (prepared by one lane, read back from LDS).
struct __align__(16) SepCol {
    WinCol w;    // the column's z mapping at the plane
    double pos;  // in-plane position where the column's rays cross the plane
};

// One wave handles 64*KZ voxels of one (x, y) column, lane + 64*q for q < KZ.
// For each view and each candidate detector column a (wave-uniform), the
// rays of column a meet the voxel's plane on a line along z where row b sits
// at zk + tz*b relative to the voxel; the lane sums hat(zk + tz*b) * data over
// the rows with |zk + tz*b| < 1 and weights the sum by the in-plane hat of
// the column.  PART 0: x-major rays on plane x = i (in-plane offset along y);
// PART 1: y-major rays on plane y = j (offset along x).
// HALF: lanes 0-31 and 32-63 hold two different j (the candidate column
// range is the union of both halves' ranges).
// The candidate columns go in batches of 32: lane c of each half works out
// column a0 + c at its half's plane (ray parameter, in-plane position, z
// mapping of the detector rows) and whether it reaches the half's row, and
// keeps it in the wave's LDS records (rec[64]: half h at 32 h); the wave then
// walks the columns that reach either half, in increasing order, each half
// reading its own record.  One lane per column and half does the set-up and
// the column descriptors arrive in one round of loads.  LDS operations of a
// wave complete in order, so the records written are seen by the reads that
// follow, and the next batch's writes follow this batch's reads.
template <int PART, int KZ, int NP, typename PT, bool HALF>
__device__ __forceinline__ void bp_part(const SepView &S, const ColD *__restrict__ cv,
                                        const PT *base0, const PT *base1, int i, int j, int nu, int nv,
                                        double zw0, const float (&u)[KZ], float (&pv)[NP][KZ], SepCol *rec) {
    const float fi = (float)i, fj = (float)j;
    float c1, c2;
    if (PART == 0) {
        c1 = column_coord(S, fi, fj - 1.f);
        c2 = column_coord(S, fi, fj + 1.f);
    } else {
        c1 = column_coord(S, fi - 1.f, fj);
        c2 = column_coord(S, fi + 1.f, fj);
    }
    int alo = (int)floorf(fminf(c1, c2) - 0.01f);
    int ahi = (int)ceilf(fmaxf(c1, c2) + 0.01f);
    alo = max(alo, 0);
    ahi = min(ahi, nu - 1);
    if (HALF) {
        alo = min(__builtin_amdgcn_readlane(alo, 0), __builtin_amdgcn_readlane(alo, 32));
        ahi = max(__builtin_amdgcn_readlane(ahi, 0), __builtin_amdgcn_readlane(ahi, 32));
    } else {
        alo = __builtin_amdgcn_readfirstlane(alo);
        ahi = __builtin_amdgcn_readfirstlane(ahi);
    }
    if (alo > ahi) return;
    // distance of the plane from the source along the major axis
    const double dm = (PART == 0) ? (double)i - S.sx : (double)j - S.sy;
    const double inv_dm = 1.0 / dm;
    const double own = (PART == 0) ? (double)j : (double)i;  // the lane's row on the plane
    const int lane = threadIdx.x & 63, h = lane >> 5;
    for (int a0 = alo; a0 <= ahi; a0 += 32) {
        const int a = a0 + (lane & 31);
        bool ok = false;
        if (a <= ahi) {
            const ColD &C = cv[a];
            const double tau = dm * ((PART == 0) ? C.rdx : C.rdy);  // ray parameter at the plane
            SepCol R;
            R.pos = (PART == 0) ? fma(tau, C.dy, S.sy) : fma(tau, C.dx, S.sx);
            // row spacing along z, z of row 0, 1 / spacing at the plane
            R.w = win_col(fma(tau, S.dz0, S.sz), tau * S.vz, ((PART == 0) ? C.dxv : C.dyv) * inv_dm, zw0);
            ok = C.axis == PART && 1.f - (float)fabs(R.pos - own) > 0.f && tau >= 0.0 && tau <= 1.0;
            if (ok) rec[lane] = R;
        }
        const unsigned long long m = __ballot(ok);
        unsigned cm = (unsigned)m | (unsigned)(m >> 32);
        __builtin_amdgcn_wave_barrier();
        while (cm) {
            const int c = __builtin_ctz(cm);
            cm &= cm - 1;
            if ((m >> (32 * h + c)) & 1ull) {
                const SepCol R = rec[32 * h + c];
                const float wp = 1.f - (float)fabs(R.pos - own);
                const long ac = a0 + c;
                const PT *col0 = base0 + ac * nv;
                const PT *col1 = (NP > 1) ? base1 + ac * nv : nullptr;
                float sums[NP][KZ];
                bp_column_sums<KZ, NP, PT>(col0, col1, nv, R.w, u, sums);
#pragma unroll
                for (int q = 0; q < KZ; ++q) {
                    pv[0][q] = fmaf(wp, sums[0][q], pv[0][q]);
                    if (NP > 1) pv[NP - 1][q] = fmaf(wp, sums[NP - 1][q], pv[NP - 1][q]);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Blocked variant of bp_part: the wave covers BI x BJ rows (i, j).  A plane
// (x = i for PART 0, y = j for PART 1) is shared by the block's rows lying in
// it, so each column's detector-row sums are formed once per plane and
// weighted into every row the column reaches (the in-plane hat 1 - |off|).
// Same arithmetic per (voxel, column) as bp_part.  ZS (grids with more than
// one z chunk per row): [zw0, zw1] is the wave's z range, and planes and
// columns whose detector rows stay more than a voxel away from it are
// skipped (tall volumes, where a view's cone covers part of the height).
template <int PART, int KZ, int NP, typename PT, int BI, int BJ, bool ZS>
__device__ __forceinline__ void bp_part_blk(const SepView &S, const ColD *__restrict__ cv, const PT *base0,
                                            const PT *base1, int i0, int j0, int nu, int nv,
                                            const float (&u)[KZ], double zw0, double zw1,
                                            float (&pv)[NP][BI * BJ][KZ]) {
    constexpr int NPL = PART == 0 ? BI : BJ;  // planes in the block
    constexpr int NR = PART == 0 ? BJ : BI;   // rows per plane
    const int r0 = PART == 0 ? j0 : i0;
#pragma unroll
    for (int pl = 0; pl < NPL; ++pl) {
        const int P = (PART == 0 ? i0 : j0) + pl;
        // distance of the plane from the source along the major axis
        const double dm = (double)P - (PART == 0 ? S.sx : S.sy);
        if (ZS) {
            // rows 0 and nv-1 lie at z = s_z + tau dz0 and s_z + tau dzn at the
            // plane, tau = dm / D over the view's columns of this part: if even
            // the extremes stay a voxel away from the wave's z range, skip the plane
            const double ta = dm * (PART == 0 ? S.r0lo : S.r1lo), tb = dm * (PART == 0 ? S.r0hi : S.r1hi);
            const double dzn = fma(S.vz, (double)(nv - 1), S.dz0);
            const double z1 = fma(ta, S.dz0, S.sz), z2 = fma(tb, S.dz0, S.sz);
            const double z3 = fma(ta, dzn, S.sz), z4 = fma(tb, dzn, S.sz);
            if (fmax(fmax(z1, z2), fmax(z3, z4)) <= zw0 - 1.0 || fmin(fmin(z1, z2), fmin(z3, z4)) >= zw1 + 1.0)
                continue;
        }
        const double inv_dm = 1.0 / dm;
        const float fp = (float)P, flo = (float)(r0 - 1), fhi = (float)(r0 + NR);
        const float c1 = PART == 0 ? column_coord(S, fp, flo) : column_coord(S, flo, fp);
        const float c2 = PART == 0 ? column_coord(S, fp, fhi) : column_coord(S, fhi, fp);
        int alo = (int)floorf(fminf(c1, c2) - 0.01f);
        int ahi = (int)ceilf(fmaxf(c1, c2) + 0.01f);
        alo = __builtin_amdgcn_readfirstlane(max(alo, 0));
        ahi = __builtin_amdgcn_readfirstlane(min(ahi, nu - 1));
        for (int a = alo; a <= ahi; ++a) {
            const ColD C = cv[a];
            if (C.axis != PART) continue;
            const double tau = dm * (PART == 0 ? C.rdx : C.rdy);  // ray parameter at the plane
            if (tau < 0.0 || tau > 1.0) continue;
            const double pos = PART == 0 ? fma(tau, C.dy, S.sy) : fma(tau, C.dx, S.sx);  // in-plane position
            float w[NR];
            bool any = false;
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                w[r] = 1.f - (float)fabs(pos - (double)(r0 + r));
                any |= w[r] > 0.f;
            }
            if (!any) continue;
            const double tz = tau * S.vz;                                // row spacing along z at the plane
            const double zc = fma(tau, S.dz0, S.sz);                     // z of row 0 at the plane
            // the column's rows span [zc, zc + (nv-1) tz] at the plane: no
            // voxel of the wave within one voxel of it, no contribution
            const double zend = fma(tz, (double)(nv - 1), zc);
            if (ZS && (fmax(zc, zend) <= zw0 - 1.0 || fmin(zc, zend) >= zw1 + 1.0)) continue;
            const double rtz = (PART == 0 ? C.dxv : C.dyv) * inv_dm;     // 1 / tz
            const PT *col0 = base0 + (long)a * nv;
            const PT *col1 = (NP > 1) ? base1 + (long)a * nv : nullptr;
            float sums[NP][KZ];
            bp_column_sums<KZ, NP, PT>(col0, col1, nv, win_col(zc, tz, rtz, zw0), u, sums);
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                if (!(w[r] > 0.f)) continue;
                const int idx = PART == 0 ? pl * BJ + r : r * BJ + pl;
#pragma unroll
                for (int q = 0; q < KZ; ++q) {
                    pv[0][idx][q] = fmaf(w[r], sums[0][q], pv[0][idx][q]);
                    if (NP > 1) pv[NP - 1][idx][q] = fmaf(w[r], sums[NP - 1][q], pv[NP - 1][idx][q]);
                }
            }
        }
    }
}

// Back-projector over BI x BJ blocks of rows: wave -> (block, z chunk), lane
// -> z = zc_id * 64 KZ + 64 q + lane.  Views and chunks as k_backproject_sep.
template <int KZ, int NP, typename OT, typename PT, int BI, int BJ, bool ZS>
__global__ __launch_bounds__(256) void k_backproject_blk(const PT *__restrict__ pt0, const PT *__restrict__ pt1,
                                                         OT *__restrict__ vol0, OT *__restrict__ vol1,
                                                         float *__restrict__ part0, float *__restrict__ part1,
                                                         const SepView *__restrict__ sep,
                                                         const ColD *__restrict__ cols,
                                                         const uint8_t *__restrict__ axis, int nx, int ny, int nz,
                                                         int nu, int nv, int nviews_sub, int view0, int view_step,
                                                         int per_chunk) {
    constexpr int NB = BI * BJ;
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int zchunks = (nz + 64 * KZ - 1) / (64 * KZ);
    const int nbi = (nx + BI - 1) / BI;
    const int zc_id = wave % zchunks;
    const int blk = wave / zchunks;
    const int i0 = (blk % nbi) * BI, j0 = (blk / nbi) * BJ;
    if (j0 >= ny) return;  // whole wave; no barrier below
    double kd[KZ];
#pragma unroll
    for (int q = 0; q < KZ; ++q) kd[q] = (double)(zc_id * 64 * KZ + q * 64 + lane);
    const double zw0 = (double)(zc_id * 64 * KZ), zw1 = zw0 + (double)(64 * KZ - 1);
    float u[KZ];  // z - zw0 of the lane's voxels
#pragma unroll
    for (int q = 0; q < KZ; ++q) u[q] = (float)(q * 64 + lane);
    // per-view partial sums in FP32, summed over views in FP64
    double acc[NP][NB][KZ];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int q = 0; q < KZ; ++q) acc[p][b][q] = 0.0;

    const int vbeg = blockIdx.y * per_chunk;
    const int vend = min(nviews_sub, vbeg + per_chunk);
    for (int vl = vbeg; vl < vend; ++vl) {
        float pv[NP][NB][KZ];
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int q = 0; q < KZ; ++q) pv[p][b][q] = 0.f;
        const int v = view0 + vl * view_step;
        const SepView S = sep[v];
        const ColD *cv = cols + (long)v * nu;
        const PT *base0 = pt0 + (long)vl * nu * nv;
        const PT *base1 = (NP > 1) ? pt1 + (long)vl * nu * nv : nullptr;
        if (S.flags & 1) bp_part_blk<0, KZ, NP, PT, BI, BJ, ZS>(S, cv, base0, base1, i0, j0, nu, nv, u, zw0, zw1, pv);
        if (S.flags & 2) bp_part_blk<1, KZ, NP, PT, BI, BJ, ZS>(S, cv, base0, base1, i0, j0, nu, nv, u, zw0, zw1, pv);
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int q = 0; q < KZ; ++q) acc[p][b][q] += (double)pv[p][b][q];
    }
    const long nvox = (long)nx * ny * nz;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int i = i0 + b / BJ, j = j0 + b % BJ;
#pragma unroll
        for (int q = 0; q < KZ; ++q) {
            const int k = (int)kd[q];
            if (i < nx && j < ny && k < nz) {
                const long o = ((long)k * ny + j) * nx + i;
                if (gridDim.y == 1) {
                    store_f(vol0, o, (float)acc[0][b][q]);
                    if (NP > 1) store_f(vol1, o, (float)acc[NP - 1][b][q]);
                } else {
                    part0[blockIdx.y * nvox + o] = (float)acc[0][b][q];
                    if (NP > 1) part1[blockIdx.y * nvox + o] = (float)acc[NP - 1][b][q];
                }
            }
        }
    }
}

// Views [chunk*per, min(nviews_sub, (chunk+1)*per)) with chunk = blockIdx.y.
// With one chunk the result goes straight to vol0/vol1 (type OT); with more,
// each chunk writes FP32 partial volumes part0/part1 + chunk * nvox, summed
// afterwards in a fixed order (deterministic).
template <int KZ, int NP, typename OT, typename PT, bool HALF>
__global__ __launch_bounds__(256) void k_backproject_sep(const PT *__restrict__ pt0, const PT *__restrict__ pt1,
                                                         OT *__restrict__ vol0, OT *__restrict__ vol1,
                                                         float *__restrict__ part0, float *__restrict__ part1,
                                                         const SepView *__restrict__ sep,
                                                         const ColD *__restrict__ cols,
                                                         const uint8_t *__restrict__ axis, int nx, int ny, int nz,
                                                         int nu, int nv, int nviews_sub, int view0, int view_step,
                                                         int per_chunk) {
    __shared__ SepCol recs[4][64];
    SepCol *rec = recs[threadIdx.x >> 6];
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    // HALF (nz <= 32, KZ = 1): a wave covers z = lane % 32 of two rows
    // j = 2 jp and 2 jp + 1; otherwise z = zc_id * 64 KZ + 64 q + lane of one row
    const int zchunks = HALF ? 1 : (nz + 64 * KZ - 1) / (64 * KZ);
    const int zc_id = wave % zchunks;
    const int ij = wave / zchunks;
    const int i = ij % nx;
    const int jw = HALF ? 2 * (ij / nx) : ij / nx;  // the wave's first row
    if (jw >= ny) return;  // whole wave; no barrier below
    const int j = HALF ? jw + (lane >> 5) : jw;
    double kd[KZ];
#pragma unroll
    for (int q = 0; q < KZ; ++q) kd[q] = HALF ? (double)(lane & 31) : (double)(zc_id * 64 * KZ + q * 64 + lane);
    // the wave's first z and the lanes' offsets from it
    const double zw0 = HALF ? 0.0 : (double)(zc_id * 64 * KZ);
    float u[KZ];
#pragma unroll
    for (int q = 0; q < KZ; ++q) u[q] = HALF ? (float)(lane & 31) : (float)(q * 64 + lane);
    // per-view partial sums in FP32, summed over views in FP64
    double acc[NP][KZ];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int q = 0; q < KZ; ++q) acc[p][q] = 0.0;

    const int vbeg = blockIdx.y * per_chunk;
    const int vend = min(nviews_sub, vbeg + per_chunk);
    for (int vl = vbeg; vl < vend; ++vl) {
        float pv[NP][KZ];
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int q = 0; q < KZ; ++q) pv[p][q] = 0.f;
        const int v = view0 + vl * view_step;
        const SepView S = sep[v];
        const ColD *cv = cols + (long)v * nu;
        const PT *base0 = pt0 + (long)vl * nu * nv;
        const PT *base1 = (NP > 1) ? pt1 + (long)vl * nu * nv : nullptr;
        if (S.flags & 1) bp_part<0, KZ, NP, PT, HALF>(S, cv, base0, base1, i, j, nu, nv, zw0, u, pv, rec);
        if (S.flags & 2) bp_part<1, KZ, NP, PT, HALF>(S, cv, base0, base1, i, j, nu, nv, zw0, u, pv, rec);
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int q = 0; q < KZ; ++q) acc[p][q] += (double)pv[p][q];
    }
    const long nvox = (long)nx * ny * nz;
#pragma unroll
    for (int q = 0; q < KZ; ++q) {
        const int k = (int)kd[q];
        if (k < nz && j < ny) {
            const long o = ((long)k * ny + j) * nx + i;
            if (gridDim.y == 1) {
                store_f(vol0, o, (float)acc[0][q]);
                if (NP > 1) store_f(vol1, o, (float)acc[NP - 1][q]);
            } else {
                part0[blockIdx.y * nvox + o] = (float)acc[0][q];
                if (NP > 1) part1[blockIdx.y * nvox + o] = (float)acc[NP - 1][q];
            }
        }
    }
}

template <typename OT>
__global__ void k_sum_chunks(const float *__restrict__ part, OT *__restrict__ out, long nvox, int nchunks) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < nvox; i += (long)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int c = 0; c < nchunks; ++c) acc += (double)part[c * nvox + i];
        store_f(out, i, (float)acc);
    }
}

// row block of the separable back-projector's waves (nz > 32)
#ifndef MGCT_BP_BI
#define MGCT_BP_BI 2
#endif
#ifndef MGCT_BP_BJ
#define MGCT_BP_BJ 2
#endif
#ifndef MGCT_BP_KZMAX
#define MGCT_BP_KZMAX 2
#endif
#ifndef MGCT_BP_HALF_MAXNZ
#define MGCT_BP_HALF_MAXNZ 32  // grids at most this deep use the paired-row kernel
#endif
#ifndef MGCT_BP_MIN_VIEWS
#define MGCT_BP_MIN_VIEWS 2    // fewest views per view chunk
#endif
#ifndef MGCT_BP_PLANE
#define MGCT_BP_PLANE 1        // grids deeper than MGCT_BP_HALF_MAXNZ: plane-blocked kernel (0: 2 x 2 row blocks)
#endif
constexpr int kBpBI = MGCT_BP_BI, kBpBJ = MGCT_BP_BJ;

// ------------------------------------------ plane-blocked back-projector --
//
// One wave per (plane, kPlRows in-plane rows, 64 KZ z values) of one major
// axis: PART 0 waves own the plane x = i with rows y = j0 .. j0+7 and take the
// views' x-major columns, PART 1 waves own y = j with rows x = i0 .. i0+7 and
// the y-major columns (blockIdx.z).  A column crossing the plane at in-plane
// position pos reaches exactly the rows floor(pos) and floor(pos) + 1, both
// wave-uniform, so the column's detector-row sums for the wave's z values
// (bp_column_sums) are formed once and added, with the in-plane hat weights
// 1 - f and f (f = pos - floor(pos)), to those two rows.  The rows are picked
// by a runtime index, so the sums live in LDS slots private to each lane (no
// other lane touches them: no barriers), with two spare rows for the taps
// that fall just outside the block.  The slot updates are plain LDS
// read-add-writes (exact, as the slots are lane-private; the LDS atomic add
// measured about five times slower here).  The parts write separate partial
// volumes, summed with the view chunks afterwards.  Per voxel and view this
// forms about 1.6 column sums against 2.5 for the 2 x 2 row blocks
// (k_backproject_blk, kept for comparison builds).
//
// The views go in groups of kBpGroup: the candidate columns of all the
// group's views at the wave's plane form one list, and the per-column set-up
// (ray parameter, in-plane position, z mapping, in FP64) runs one column per
// lane over that list, so a batch of 64 lanes serves several views instead of
// the dozen or so columns one view has at one plane.  The slots collect the
// whole group's sums in FP32 and are added to FP64 registers (and cleared)
// once per group.
#ifndef MGCT_BP_PLROWS
#define MGCT_BP_PLROWS 8
#endif
#ifndef MGCT_BP_GROUP
#define MGCT_BP_GROUP 16
#endif
constexpr int kPlRows = MGCT_BP_PLROWS;
constexpr int kPlSlots = kPlRows + 2;
constexpr int kBpGroup = MGCT_BP_GROUP;

// What the column loop needs of one column at the wave's plane (prepared
// by one lane, read back by the whole wave from LDS).
struct __align__(16) PlCol {
    WinCol w;      // the column's z mapping at the plane
    float whi;     // in-plane hat weight of the upper row
    int rl;        // block row of the lower tap (-1 .. kPlRows-1)
    uint32_t off;  // element offset of the column's first detector row in the stack
    int r0;        // w.R0 as an integer
};

// Column records per batch and the waves per SIMD the registers must allow,
// by variant.  The single-output variant for grids of one 128-deep z chunk
// (KZ = 2, no z-range test) runs 6 waves per SIMD: its records then go in
// batches of 32 so that slots and records fit 6 blocks per CU in LDS, and its
// registers are held to 80.  The others keep batches of 64 and 5 waves.
template <int KZ, int NP, bool ZS> constexpr bool bp_pl_six() { return KZ == 2 && NP == 1 && !ZS; }
template <int KZ, int NP, bool ZS> constexpr int bp_pl_batch() { return bp_pl_six<KZ, NP, ZS>() ? 32 : 64; }
template <int KZ, int NP, bool ZS> constexpr int bp_pl_minw() {
    return NP > 1 ? 1 : (bp_pl_six<KZ, NP, ZS>() ? 6 : 5);
}

__device__ __forceinline__ float uniform_f(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}

// The candidate columns of one view at plane P (those whose rays can cross
// the in-plane rows r0-1 .. r0+kPlRows), as a range [lo, lo + n); n = 0 when
// the view has no columns of this axis or (ZS) its extreme rows stay a voxel
// away from the wave's z range [zw0, zw1] at this plane.
template <int PART, bool ZS>
__device__ __forceinline__ void bp_view_range(const SepView &S, int P, int r0, int nu, int nv, double zw0,
                                              double zw1, int &lo, int &n) {
    lo = 0;
    n = 0;
    if (!(S.flags & (PART == 0 ? 1 : 2))) return;
    const double dm = (double)P - (PART == 0 ? S.sx : S.sy);  // plane's distance from the source
    if (ZS) {
        const double ta = dm * (PART == 0 ? S.r0lo : S.r1lo), tb = dm * (PART == 0 ? S.r0hi : S.r1hi);
        const double dzn = fma(S.vz, (double)(nv - 1), S.dz0);
        const double z1 = fma(ta, S.dz0, S.sz), z2 = fma(tb, S.dz0, S.sz);
        const double z3 = fma(ta, dzn, S.sz), z4 = fma(tb, dzn, S.sz);
        if (fmax(fmax(z1, z2), fmax(z3, z4)) <= zw0 - 1.0 || fmin(fmin(z1, z2), fmin(z3, z4)) >= zw1 + 1.0) return;
    }
    const float fp = (float)P, flo = (float)(r0 - 1), fhi = (float)(r0 + kPlRows);
    const float c1 = PART == 0 ? column_coord(S, fp, flo) : column_coord(S, flo, fp);
    const float c2 = PART == 0 ? column_coord(S, fp, fhi) : column_coord(S, fhi, fp);
    const int alo = max((int)floorf(fminf(c1, c2) - 0.01f), 0);
    const int ahi = min((int)ceilf(fmaxf(c1, c2) + 0.01f), nu - 1);
    lo = alo;
    n = max(ahi - alo + 1, 0);
}

// The column walk, software-pipelined: the next column's record is read and
// its detector-row loads issued before the current column's sums are formed,
// so each wave keeps two columns' loads in flight.  Columns whose rows lie at
// least half a voxel apart along z (|1/tz| < 2, the usual case) take a fixed
// window of 4 rows (it holds every row within one voxel of z; the hat weights
// of the others are 0; a 3-row window where |1/tz| < 1.5 measured slower); the
// others re-read their record and take the variable window of
// bp_column_sums.  Needs nv >= 4.
template <int KZ, int NP> struct BpFetch {
    float v[NP][KZ][4];  // the window's rows
    float d0[KZ];        // hat argument of the window's first row
    float tzh, whi;
    int rl, l;           // slot row, record index (wave-uniform)
    bool w4;             // the 4-row window applies (wave-uniform)
};

template <int KZ, int NP, typename PT>
__device__ __forceinline__ void bp_fetch(BpFetch<KZ, NP> &F, const PlCol *rec, int l, const PT *pt0,
                                         const PT *pt1, int nv, const float (&u)[KZ]) {
    // the record is the same in every lane: the column's address and the
    // window test go to scalar registers, the slot row stays a vector value
    // (one lane read fewer); the window's first row as an integer sum
    PlCol R = rec[l];
    const uint32_t off = __builtin_amdgcn_readfirstlane(R.off);
    F.rl = R.rl;
    F.l = l;
    R.w.rtz = uniform_f(R.w.rtz);
    F.w4 = fabsf(R.w.rtz) < 2.f;
    F.tzh = R.w.tzh;
    F.whi = R.whi;
    const float hi = (float)(nv - 4) - R.w.R0;
#pragma unroll
    for (int q = 0; q < KZ; ++q) {
        float dl;
        win_start(R.w, u[q], hi, dl, F.d0[q]);
        const uint32_t bs = (uint32_t)((int)dl + R.r0);  // dl is an integer
        load_win<4>(pt0 + off, bs, F.v[0][q]);
        if (NP > 1) load_win<4>(pt1 + off, bs, F.v[NP - 1][q]);
    }
}

template <int KZ, int NP, typename PT>
__device__ __forceinline__ void bp_finish(const BpFetch<KZ, NP> &F, const PlCol *rec, const PT *pt0,
                                          const PT *pt1, int nv, const float (&u)[KZ], float *slot) {
    float sums[NP][KZ];
    if (F.w4) {
#pragma unroll
        for (int q = 0; q < KZ; ++q) {
            float s0 = 0.f, s1 = 0.f;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const float h = hat(t == 0 ? F.d0[q] : fmaf((float)t, F.tzh, F.d0[q]));
                s0 = fmaf(h, F.v[0][q][t], s0);
                if (NP > 1) s1 = fmaf(h, F.v[NP - 1][q][t], s1);
            }
            sums[0][q] = s0;
            if (NP > 1) sums[NP - 1][q] = s1;
        }
    } else {
        PlCol R = rec[F.l];
        const uint32_t off = __builtin_amdgcn_readfirstlane(R.off);
        R.w.rtz = uniform_f(R.w.rtz);
        bp_column_sums<KZ, NP, PT>(pt0 + off, (NP > 1) ? pt1 + off : nullptr, nv, R.w, u, sums);
    }
    float *sl = slot + (F.rl + 1) * KZ * 64;
    const float whi = F.whi, wlo = 1.f - whi;
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int q = 0; q < KZ; ++q) {
            float *e0 = sl + (p * kPlSlots * KZ + q) * 64, *e1 = sl + ((p * kPlSlots + 1) * KZ + q) * 64;
            *e0 = fmaf(wlo, sums[p][q], *e0);
            *e1 = fmaf(whi, sums[p][q], *e1);
        }
}

// Walks the set bits of m (increasing), two columns in flight.  The last
// prefetch repeats the current column (its loads are in bounds) and is
// dropped.
template <int KZ, int NP, typename PT>
__device__ __forceinline__ void bp_walk(unsigned long long m, const PlCol *rec, const PT *pt0, const PT *pt1, int nv,
                                        const float (&u)[KZ], float *slot) {
    if (!m) return;
    int la = __builtin_ctzll(m);
    m &= m - 1;
    BpFetch<KZ, NP> A, B;
    bp_fetch<KZ, NP, PT>(A, rec, la, pt0, pt1, nv, u);
    while (true) {
        bool more = m != 0;
        const int lb = more ? __builtin_ctzll(m) : la;
        m &= m - 1;
        bp_fetch<KZ, NP, PT>(B, rec, lb, pt0, pt1, nv, u);
        bp_finish<KZ, NP, PT>(A, rec, pt0, pt1, nv, u, slot);
        if (!more) break;
        more = m != 0;
        la = more ? __builtin_ctzll(m) : lb;
        m &= m - 1;
        bp_fetch<KZ, NP, PT>(A, rec, la, pt0, pt1, nv, u);
        bp_finish<KZ, NP, PT>(B, rec, pt0, pt1, nv, u, slot);
        if (!more) break;
    }
}

// One group of views [vg0, vg0 + kBpGroup) n [.., vend) at the wave's plane:
// sums into the slots.
template <int PART, int KZ, int NP, typename PT, bool ZS>
__device__ __forceinline__ void bp_plane_group(const SepView *__restrict__ sep, const ColD *__restrict__ cols,
                                               const PT *__restrict__ pt0, const PT *__restrict__ pt1, int P,
                                               int r0, int nu, int nv, int vg0, int vend, int view0,
                                               int view_step, const float (&u)[KZ], double zw0, double zw1,
                                               float *slot, PlCol *rec) {
    const int lane = threadIdx.x & 63;
    // lane g < kBpGroup: the candidate range of view vg0 + g
    int lo = 0, n = 0;
    if (lane < kBpGroup && vg0 + lane < vend)
        bp_view_range<PART, ZS>(sep[view0 + (vg0 + lane) * view_step], P, r0, nu, nv, zw0, zw1, lo, n);
    // the group's ranges one after the other: candidate c < tot belongs to the
    // last view g with start[g] <= c, column c + shift[g]
    int start[kBpGroup], shift[kBpGroup];
    int tot = 0;
#pragma unroll
    for (int g = 0; g < kBpGroup; ++g) {
        start[g] = tot;
        shift[g] = __builtin_amdgcn_readlane(lo, g) - tot;
        tot += __builtin_amdgcn_readlane(n, g);
    }
    // Batches of RB candidates (64, or 32 in the 6-wave variant): lane l < RB
    // works out candidate c0 + l at this plane (ray parameter, in-plane
    // position and rows, z mapping of the detector rows), whether it reaches
    // the block, and keeps the result in the wave's LDS records; the wave
    // then walks the columns that do (the ballot's set bits, in increasing
    // order), reading each record back with broadcast loads.  LDS operations
    // of a wave complete in order, so a record written by one lane is seen by
    // the next read, and the next batch's writes follow this batch's reads.
    constexpr int RB = bp_pl_batch<KZ, NP, ZS>();
    for (int c0 = 0; c0 < tot; c0 += RB) {
        const int c = c0 + lane;
        bool ok = false;
        if (lane < RB && c < tot) {
            int g = 0, sh = shift[0];
#pragma unroll
            for (int t = 1; t < kBpGroup; ++t)
                if (c >= start[t]) {
                    g = t;
                    sh = shift[t];
                }
            const int vl = vg0 + g;
            const int v = view0 + vl * view_step;
            const int a = c + sh;
            const SepView &S = sep[v];
            const ColD &C = cols[(long)v * nu + a];
            const double dm = (double)P - (PART == 0 ? S.sx : S.sy);
            const double tau = dm * (PART == 0 ? C.rdx : C.rdy);                         // ray parameter at the plane
            const double pos = PART == 0 ? fma(tau, C.dy, S.sy) : fma(tau, C.dx, S.sx);  // in-plane position
            const double fl = fmin(fmax(floor(pos), -1e9), 1e9);
            const double tz = tau * S.vz;             // row spacing along z at the plane
            const double zc = fma(tau, S.dz0, S.sz);  // z of row 0 at the plane
            PlCol R;
            R.rl = (int)fl - r0;
            R.w = win_col(zc, tz, (PART == 0 ? C.dxv : C.dyv) / dm, zw0);
            R.r0 = (int)R.w.R0;
            R.whi = (float)(pos - fl);
            R.off = (uint32_t)(((long)vl * nu + a) * nv);
            ok = C.axis == PART && tau >= 0.0 && tau <= 1.0 && R.rl >= -1 && R.rl < kPlRows;
            if (ZS && ok) {
                const double zend = fma(tz, (double)(nv - 1), zc);
                ok = !(fmax(zc, zend) <= zw0 - 1.0 || fmin(zc, zend) >= zw1 + 1.0);
            }
            if (ok) rec[lane] = R;
        }
        unsigned long long m = __ballot(ok);
        __builtin_amdgcn_wave_barrier();
        if (nv >= 4) {
            bp_walk<KZ, NP, PT>(m, rec, pt0, pt1, nv, u, slot);
            m = 0;
        }
        while (m) {
            const int l = __builtin_ctzll(m);
            m &= m - 1;
            PlCol R = rec[l];
            // the record is the same in every lane: scalar column address,
            // slot row and window-width branch
            const uint32_t off = __builtin_amdgcn_readfirstlane(R.off);
            const int rl = __builtin_amdgcn_readfirstlane(R.rl);
            R.w.rtz = uniform_f(R.w.rtz);
            float *sl = slot + (rl + 1) * KZ * 64;
            float old[NP][2][KZ];
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int q = 0; q < KZ; ++q) {
                    old[p][0][q] = sl[(p * kPlSlots * KZ + q) * 64];
                    old[p][1][q] = sl[((p * kPlSlots + 1) * KZ + q) * 64];
                }
            const float whi = R.whi, wlo = 1.f - whi;
            const PT *col0 = pt0 + off;
            const PT *col1 = (NP > 1) ? pt1 + off : nullptr;
            float sums[NP][KZ];
            bp_column_sums<KZ, NP, PT>(col0, col1, nv, R.w, u, sums);
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int q = 0; q < KZ; ++q) {
                    sl[(p * kPlSlots * KZ + q) * 64] = fmaf(wlo, sums[p][q], old[p][0][q]);
                    sl[((p * kPlSlots + 1) * KZ + q) * 64] = fmaf(whi, sums[p][q], old[p][1][q]);
                }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

template <int PART, int KZ, int NP, typename PT, bool ZS>
__device__ __forceinline__ void bp_plane_wave(const PT *__restrict__ pt0, const PT *__restrict__ pt1,
                                              float *__restrict__ part, long np_stride, float *slot, PlCol *rec,
                                              const SepView *__restrict__ sep, const ColD *__restrict__ cols,
                                              int nx, int ny, int nz, int nu, int nv, int nviews_sub, int view0,
                                              int view_step, int per_chunk, int nchunks) {
    const int lane = threadIdx.x & 63;
    const int nplanes = PART == 0 ? nx : ny, nrows = PART == 0 ? ny : nx;
    const int nrb = (nrows + kPlRows - 1) / kPlRows;
    const int zchunks = (nz + 64 * KZ - 1) / (64 * KZ);
    // block -> (4 consecutive planes, row block, z chunk); wave -> plane
    const int zc_id = blockIdx.x % zchunks;
    const int rb = (blockIdx.x / zchunks) % nrb;
    const int P0 = blockIdx.x / zchunks / nrb * 4;
    if (P0 >= nplanes) return;  // whole block, before any barrier
    const int P = P0 + (threadIdx.x >> 6);
    const bool live = P < nplanes;
    const int r0 = rb * kPlRows;
    double kd[KZ];
#pragma unroll
    for (int q = 0; q < KZ; ++q) kd[q] = (double)(zc_id * 64 * KZ + q * 64 + lane);
    const double zw0 = (double)(zc_id * 64 * KZ), zw1 = zw0 + (double)(64 * KZ - 1);
    float u[KZ];  // z - zw0 of the lane's voxels
#pragma unroll
    for (int q = 0; q < KZ; ++q) u[q] = (float)(q * 64 + lane);
#pragma unroll
    for (int t = 0; t < NP * kPlSlots * KZ; ++t) slot[t * 64] = 0.f;
    double acc[NP][kPlRows][KZ];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int r = 0; r < kPlRows; ++r)
#pragma unroll
            for (int q = 0; q < KZ; ++q) acc[p][r][q] = 0.0;
    const int vbeg = blockIdx.y * per_chunk;
    const int vend = min(nviews_sub, vbeg + per_chunk);
    for (int vg0 = vbeg; vg0 < vend; vg0 += kBpGroup) {
        // The block's waves (neighbouring planes: nearly the same detector
        // columns and rows) start each group together, so that their reads
        // of the group's detector data meet in the caches.
        __syncthreads();
        if (!live) continue;
        bp_plane_group<PART, KZ, NP, PT, ZS>(sep, cols, pt0, pt1, P, r0, nu, nv, vg0, vend, view0, view_step, u, zw0,
                                             zw1, slot, rec);
        // the group's sums into FP64, slots cleared (spare rows too)
#pragma unroll
        for (int p = 0; p < NP; ++p) {
#pragma unroll
            for (int r = 0; r < kPlRows; ++r)
#pragma unroll
                for (int q = 0; q < KZ; ++q) {
                    float *e = slot + ((p * kPlSlots + r + 1) * KZ + q) * 64;
                    acc[p][r][q] += (double)*e;
                    *e = 0.f;
                }
#pragma unroll
            for (int q = 0; q < KZ; ++q) {
                slot[((p * kPlSlots) * KZ + q) * 64] = 0.f;
                slot[((p * kPlSlots + kPlSlots - 1) * KZ + q) * 64] = 0.f;
            }
        }
    }
    const long nvox = (long)nx * ny * nz;
    float *out = part + (long)(PART * nchunks + blockIdx.y) * nvox;
#pragma unroll
    for (int r = 0; r < kPlRows; ++r) {
        const int row = r0 + r;
        const int i = PART == 0 ? P : row, j = PART == 0 ? row : P;
#pragma unroll
        for (int q = 0; q < KZ; ++q) {
            const int k = (int)kd[q];
            if (live && row < nrows && k < nz) {
                const long o = ((long)k * ny + j) * nx + i;
                out[o] = (float)acc[0][r][q];
                if (NP > 1) out[np_stride + o] = (float)acc[NP - 1][r][q];
            }
        }
    }
}

// Launch: grid (blocks of 4 planes x row blocks x z chunks, view chunks, 2 parts);
// part[] receives 2 x chunks
// partial volumes per output (the second output np_stride floats further).
// The stack's element offsets must fit 32 bits (checked by the launcher).
template <int KZ, int NP, typename PT, bool ZS>
__global__ __launch_bounds__(256, (bp_pl_minw<KZ, NP, ZS>())) void k_backproject_pl(const PT *__restrict__ pt0, const PT *__restrict__ pt1,
                                                        float *__restrict__ part, long np_stride,
                                                        const SepView *__restrict__ sep,
                                                        const ColD *__restrict__ cols, int nx, int ny, int nz, int nu,
                                                        int nv, int nviews_sub, int view0, int view_step,
                                                        int per_chunk, int nchunks) {
    __shared__ float lds[4 * NP * kPlSlots * KZ * 64];
    __shared__ PlCol recs[4][bp_pl_batch<KZ, NP, ZS>()];
    float *slot = lds + (threadIdx.x >> 6) * (NP * kPlSlots * KZ * 64) + (threadIdx.x & 63);
    PlCol *rec = recs[threadIdx.x >> 6];
    if (blockIdx.z == 0)
        bp_plane_wave<0, KZ, NP, PT, ZS>(pt0, pt1, part, np_stride, slot, rec, sep, cols, nx, ny, nz, nu, nv, nviews_sub,
                                         view0, view_step, per_chunk, nchunks);
    else
        bp_plane_wave<1, KZ, NP, PT, ZS>(pt0, pt1, part, np_stride, slot, rec, sep, cols, nx, ny, nz, nu, nv, nviews_sub,
                                         view0, view_step, per_chunk, nchunks);
}

// waves of the separable back-projector: one per two rows when nz <= 32;
// deeper grids one per (plane, kPlRows rows, 64 KZ z) of each part (both
// parts counted), or one per kBpBI x kBpBJ block of rows and 64 KZ z values
long bp_waves(const Level &L, int *kz, int np) {
    // KZ = 2 where the depth allows (the dual-output variant keeps KZ = 1:
    // its FP64 sums would take too many registers)
    int KZ = 1;
    if (MGCT_BP_KZMAX >= 2 && 2 * 64 <= L.nz && (np == 1 || !MGCT_BP_PLANE)) KZ = 2;
    if (kz) *kz = KZ;
    if (L.nz <= MGCT_BP_HALF_MAXNZ) return (long)L.nx * ((L.ny + 1) / 2);
    const long zch = (L.nz + 64 * KZ - 1) / (64 * KZ);
    if (MGCT_BP_PLANE)
        return 2 * zch * std::max((long)L.nx * ((L.ny + kPlRows - 1) / kPlRows),
                                  (long)L.ny * ((L.nx + kPlRows - 1) / kPlRows));
    return zch * ((L.nx + kBpBI - 1) / kBpBI) * ((L.ny + kBpBJ - 1) / kBpBJ);
}

#ifndef MGCT_BP_WAVES
#define MGCT_BP_WAVES 16384  // waves the view chunks aim for
#endif
// View chunks (partial volumes summed afterwards) so that about MGCT_BP_WAVES
// waves run, each over at least MGCT_BP_MIN_VIEWS views.
int bp_chunks(const Level &L, int nviews_sub, int np) {
    const long waves = bp_waves(L, nullptr, np);
    long c = (MGCT_BP_WAVES + waves - 1) / waves;
    if (c > 64) c = 64;
    if (c > nviews_sub / MGCT_BP_MIN_VIEWS) c = nviews_sub / MGCT_BP_MIN_VIEWS;
    return c < 1 ? 1 : (int)c;
}

// partial volumes per output: the view chunks, times the two parts of the
// plane-blocked kernel
static bool bp_plane(const Level &L) { return MGCT_BP_PLANE && L.nz > MGCT_BP_HALF_MAXNZ; }
static int bp_slices(const Level &L, int nviews_sub, int np) {
    return bp_chunks(L, nviews_sub, np) * (bp_plane(L) ? 2 : 1);
}

// With more than one view chunk the chunks' partial volumes are summed into
// vol0/vol1 here, unless `leave_chunks` is set (the caller then reads the
// partials itself; *nchunks_out receives the chunk count).
template <int NP, typename OT, typename PT>
static hipError_t launch_bp(const PT *pt0, const PT *pt1, OT *vol0, OT *vol1, float *part, const Level &L,
                            int view0, int view_step, int nviews_sub, hipStream_t s, bool leave_chunks = false,
                            int *nchunks_out = nullptr) {
    if (!L.separable) return hipErrorNotSupported;
    int KZ = 1;
    const long waves = bp_waves(L, &KZ, NP);
    const int nchunks = bp_chunks(L, nviews_sub, NP);
    const int nslices = bp_slices(L, nviews_sub, NP);
    const int per = (nviews_sub + nchunks - 1) / nchunks;
    const long nvox = (long)L.nx * L.ny * L.nz;
    float *part0 = part, *part1 = part ? part + (long)nslices * nvox : nullptr;
    if (nslices > 1 && !part) return hipErrorInvalidValue;
    if (bp_plane(L)) {
        // column records carry 32-bit element offsets into the stack
        if ((unsigned long long)nviews_sub * L.nu * L.nv > 0xFFFFFFFFull) return hipErrorNotSupported;
        const long zch = (L.nz + 64 * KZ - 1) / (64 * KZ);
        const long bx = zch * std::max((long)((L.nx + 3) / 4) * ((L.ny + kPlRows - 1) / kPlRows),
                                       (long)((L.ny + 3) / 4) * ((L.nx + kPlRows - 1) / kPlRows));
        dim3 grid((unsigned)bx, (unsigned)nchunks, 2);
        const long nps = (long)nslices * nvox;
#define MGCT_BPL(K, Z)                                                                                              \
    k_backproject_pl<K, NP, PT, Z><<<grid, 256, 0, s>>>(pt0, pt1, part, nps, L.d_sep, L.d_cols, L.nx, L.ny, L.nz,     \
                                                        L.nu, L.nv, nviews_sub, view0, view_step, per, nchunks)
        if (KZ == 2) {
            if (L.nz > 128) MGCT_BPL(2, true);
            else MGCT_BPL(2, false);
        } else {
            if (L.nz > 64) MGCT_BPL(1, true);
            else MGCT_BPL(1, false);
        }
#undef MGCT_BPL
    } else {
        dim3 grid((unsigned)((waves + 3) / 4), (unsigned)nchunks);
#define MGCT_BPB_Z(K, Z)                                                                                            \
    k_backproject_blk<K, NP, OT, PT, kBpBI, kBpBJ, Z><<<grid, 256, 0, s>>>(pt0, pt1, vol0, vol1, part0, part1,       \
                                                                         L.d_sep, L.d_cols, L.d_axis, L.nx, L.ny,   \
                                                                         L.nz, L.nu, L.nv, nviews_sub, view0,       \
                                                                         view_step, per)
#define MGCT_BPB(K)                                                                                                 \
    do {                                                                                                            \
        if (L.nz > 64 * (K)) MGCT_BPB_Z(K, true);                                                                   \
        else MGCT_BPB_Z(K, false);                                                                                  \
    } while (0)
#define MGCT_BP(K, H)                                                                                               \
    k_backproject_sep<K, NP, OT, PT, H><<<grid, 256, 0, s>>>(pt0, pt1, vol0, vol1, part0, part1, L.d_sep, L.d_cols,     \
                                                      L.d_axis, L.nx, L.ny, L.nz, L.nu, L.nv, nviews_sub, view0,      \
                                                      view_step, per)
        if (L.nz <= MGCT_BP_HALF_MAXNZ) {
            MGCT_BP(1, true);
        } else {
            if (KZ == 2) MGCT_BPB(2);
            else MGCT_BPB(1);
        }
#undef MGCT_BP
#undef MGCT_BPB
#undef MGCT_BPB_Z
    }
    if (nchunks_out) *nchunks_out = nslices;
    if (nslices > 1 && !leave_chunks) {
        unsigned g = (unsigned)std::min<long>((nvox + 255) / 256, 65535L * 4);
        k_sum_chunks<OT><<<g, 256, 0, s>>>(part0, vol0, nvox, nslices);
        if (NP > 1) k_sum_chunks<OT><<<g, 256, 0, s>>>(part1, vol1, nvox, nslices);
    }
    return hipGetLastError();
}

size_t backproject_scratch_bytes(const Level &L, int nviews_sub, int np) {
    const int c = bp_slices(L, nviews_sub, np);
    return c > 1 ? (size_t)c * L.vox() * sizeof(float) * np : 0;
}

hipError_t launch_backproject(const void *pt, int pt_dtype, void *vol, int vol_dtype, float *scratch, const Level &L,
                              int view0, int view_step, int nviews_sub, hipStream_t s) {
#define MGCT_LBP(OT, PT)                                                                                           \
    return launch_bp<1, OT, PT>((const PT *)pt, nullptr, (OT *)vol, nullptr, scratch, L, view0, view_step,         \
                                nviews_sub, s)
    if (vol_dtype == MGCT_F32 && pt_dtype == MGCT_F32) MGCT_LBP(float, float);
    if (vol_dtype == MGCT_BF16 && pt_dtype == MGCT_F32) MGCT_LBP(uint16_t, float);
    if (vol_dtype == MGCT_F32 && pt_dtype == MGCT_F16) MGCT_LBP(float, _Float16);
    if (vol_dtype == MGCT_BF16 && pt_dtype == MGCT_F16) MGCT_LBP(uint16_t, _Float16);
#undef MGCT_LBP
    return hipErrorInvalidValue;
}

hipError_t launch_backproject2(const float *pt0, const float *pt1, float *vol0, float *vol1, float *scratch,
                               const Level &L, int view0, int view_step, int nviews_sub, hipStream_t s,
                               int *nchunks_left) {
    return launch_bp<2, float, float>(pt0, pt1, vol0, vol1, scratch, L, view0, view_step, nviews_sub, s,
                                      nchunks_left != nullptr, nchunks_left);
}

}  // namespace mgct

namespace mgct {

// ------------------------------------------------- geometry derivative --
//
// d/d(view parameters) of sum over rays of g[ray] * (A vol)[ray], for the
// 12 values (s, d, u, v) of every view.  Same ray walk as k_project (major
// axis and plane set held fixed, the sum being piecewise smooth).  With
// D = q - s and t = (plane - s_m)/D_m, a sample's in-plane coordinates are
// p_k = s_k + t D_k, so dp_k/ds_k = 1 - t, dp_k/dq_k = t,
// dp_k/ds_m = D_k (t - 1)/D_m and dp_k/dq_m = -D_k t/D_m; the bilinear
// sample's derivative along each in-plane axis is the tap difference
// interpolated along the other axis.  The ray value is L * sum with
// L = h|D|/|D_m|.  Pixel centre q = d + ca u + cb v.
// Each block reduces its rays' 12-vectors in FP64 into one partial per block;
// k_geom_grad_sum then adds a view's partials in a fixed order.
template <typename VT>
__global__ __launch_bounds__(256) void k_geom_grad(const VT *__restrict__ vt, const float *__restrict__ cot,
                                                   const ViewIdx *__restrict__ views,
                                                   const uint8_t *__restrict__ axis, long axis_view_stride,
                                                   long axis_row_stride, int nx, int ny, int nz, int nu, int nv,
                                                   double h, double *__restrict__ partial) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int a = blockIdx.x * 4 + w;
    const int b = blockIdx.y * 64 + lane;
    const int v = blockIdx.z;
    double out[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) out[k] = 0.0;
    const float gr = (a < nu && b < nv) ? cot[((long)v * nv + b) * nu + a] : 0.f;
    if (gr != 0.f) {
        const ViewIdx &V = views[v];
        double D[3];
        const double len = ray_setup(V, nu, nv, a, b, D);
        const int m = axis[v * axis_view_stride + b * axis_row_stride + a];
        const int ia = (m == 0) ? 1 : 0;
        const double Dm = D[m], Da = D[ia], Dz = D[2];
        const double sm = V.s[m], sa = V.s[ia], sz = V.s[2];
        const double Ba = Da / Dm, Bz = Dz / Dm;
        const double Aa = sa - sm * Ba, Az = sz - sm * Bz;
        const int n_m = (m == 0) ? nx : ny, n_a = (m == 0) ? ny : nx;
        double lo = fmax(0.0, ceil(fmin(sm, sm + Dm)));
        double hi = fmin((double)(n_m - 1), floor(fmax(sm, sm + Dm)));
        clip_range(lo, hi, Aa, Ba, -1.5, n_a + 0.5);
        clip_range(lo, hi, Az, Bz, -1.5, nz + 0.5);
        if (!(fabs(Dm) > 0.0) || !isfinite(Ba) || !isfinite(Bz)) hi = lo - 1.0;
        // sums over samples: value, and per in-plane axis c the derivative
        // (index units) and its t-weighted sum
        double S = 0.0, Ga = 0.0, Gat = 0.0, Gz = 0.0, Gzt = 0.0;
        if (lo <= hi) {
            const int l0 = (int)lo, l1 = (int)hi;
            const int PY = ny + 2 * kVolPad, PZ = nz + 2 * kVolPad;
            const int Sm = (m == 0) ? PY * PZ : PZ;
            const int Sa = (m == 0) ? PZ : PY * PZ;
            // sample coordinates stepped in 32.32 fixed point as in k_project,
            // and the ray parameter t = (l - s_m) / D_m stepped by 1 / D_m (the
            // sums stay FP64)
            const double fa0 = fma((double)l0, Ba, Aa + kVolPad), fz0 = fma((double)l0, Bz, Az + kVolPad);
            const double ga0 = floor(fa0), gz0 = floor(fz0), gba = floor(Ba), gbz = floor(Bz);
            int ai = (int)ga0, zi = (int)gz0;
            uint32_t af = frac_u32(fa0 - ga0), zf = frac_u32(fz0 - gz0);
            const int bai = (int)gba, bzi = (int)gbz;
            const uint32_t baf = frac_u32(Ba - gba), bzf = frac_u32(Bz - gbz);
            const double rDm = 1.0 / Dm;
            double t = ((double)l0 - sm) * rDm;
            for (int l = l0; l <= l1; ++l) {
                const float wa = (float)af * 0x1p-32f, wz = (float)zf * 0x1p-32f;
                const uint32_t off = (uint32_t)((l + kVolPad) * Sm + ai * Sa + zi);
                const float2 r0 = load_pair(vt, off), r1 = load_pair(vt, off + Sa);
                const float q0 = fmaf(wz, r0.y - r0.x, r0.x), q1 = fmaf(wz, r1.y - r1.x, r1.x);
                const float f = fmaf(wa, q1 - q0, q0);
                const float dfa = q1 - q0;
                const float dfz = fmaf(wa, (r1.y - r1.x) - (r0.y - r0.x), r0.y - r0.x);
                S += (double)f;
                Ga += (double)dfa;
                Gat += t * (double)dfa;
                Gz += (double)dfz;
                Gzt += t * (double)dfz;
                t += rDm;
                const uint32_t na = af + baf, nz2 = zf + bzf;
                ai += bai + (na < af ? 1 : 0);
                zi += bzi + (nz2 < zf ? 1 : 0);
                af = na;
                zf = nz2;
            }
        }
        // to physical units: positions scale by h, derivatives per index unit by 1/h
        const double L = h * len / fabs(Dm);
        double ds[3] = {0, 0, 0}, dq[3] = {0, 0, 0};
        ds[ia] = (Ga - Gat) / h;
        dq[ia] = Gat / h;
        ds[2] = (Gz - Gzt) / h;
        dq[2] = Gzt / h;
        ds[m] = ((Gat - Ga) * Da + (Gzt - Gz) * Dz) / (Dm * h);
        dq[m] = -(Gat * Da + Gzt * Dz) / (Dm * h);
        double dL[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) dL[k] = D[k] / (len * fabs(Dm));
        dL[m] -= len / (Dm * fabs(Dm));
        const double ca = a - 0.5 * (nu - 1), cb = b - 0.5 * (nv - 1);
        const double gd = (double)gr;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double dys = L * ds[k] - dL[k] * S;
            const double dyq = L * dq[k] + dL[k] * S;
            out[k] = gd * dys;
            out[3 + k] = gd * dyq;
            out[6 + k] = gd * ca * dyq;
            out[9 + k] = gd * cb * dyq;
        }
    }
    // block reduction of the 12 sums (fixed order)
    __shared__ double red[12][256];
#pragma unroll
    for (int k = 0; k < 12; ++k) red[k][threadIdx.x] = out[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
#pragma unroll
            for (int k = 0; k < 12; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 12) {
        const long bpv = (long)gridDim.x * gridDim.y;
        const long blk = (long)blockIdx.y * gridDim.x + blockIdx.x;
        partial[((long)v * bpv + blk) * 12 + threadIdx.x] = red[threadIdx.x][0];
    }
}

__global__ void k_geom_grad_sum(const double *__restrict__ partial, long bpv, double *__restrict__ dviews) {
    const int v = blockIdx.x;
    if (threadIdx.x < 12) {
        double acc = 0.0;
        for (long i = 0; i < bpv; ++i) acc += partial[((long)v * bpv + i) * 12 + threadIdx.x];
        dviews[(long)v * 12 + threadIdx.x] = acc;
    }
}

size_t geom_grad_partial_bytes(const Level &L) {
    const long bpv = (long)((L.nu + 3) / 4) * ((L.nv + 63) / 64);
    return (size_t)L.nviews * bpv * 12 * sizeof(double);
}

hipError_t launch_geom_grad(const void *vt, int vt_dtype, const float *cot, double *partial, double *dviews,
                            const Level &L, hipStream_t s) {
    dim3 grid((L.nu + 3) / 4, (L.nv + 63) / 64, L.nviews);
    const long avs = L.separable ? (long)L.nu : (long)L.nu * L.nv;
    if (vt_dtype == MGCT_F32)
        k_geom_grad<float><<<grid, 256, 0, s>>>((const float *)vt, cot, L.d_views, L.d_axis, avs, L.axis_row_stride,
                                                L.nx, L.ny, L.nz, L.nu, L.nv, L.h, partial);
    else
        return hipErrorInvalidValue;
    const long bpv = (long)grid.x * grid.y;
    k_geom_grad_sum<<<L.nviews, 64, 0, s>>>(partial, bpv, dviews);
    return hipGetLastError();
}

// ---------------------------------------- general-geometry back-projector --
//
// Any detector orientation (no z-major rays).  The projector samples a ray of
// major axis m on the voxel-centre planes of m; voxel P receives from such a
// ray the product of the two hat weights of the sample on the plane through
// P.  With g = P - s and the ray direction D(a, b) = E + a u + b v (E the
// direction to pixel (0, 0)), that sample's offsets from P along the other
// in-plane axis o and along z are
//     n_o / D_m  with  n_o = g_m D_o - g_o D_m,
//     n_z / D_m  with  n_z = g_m D_z - g_z D_m,
// ratios of affine functions of the pixel (a, b).  The rays with non-zero
// weight are those inside the quadrilateral |n_o| < |D_m|, |n_z| < |D_m|
// (the image of the voxel's square on the plane).  Its centre (n_o = n_z = 0)
// is the voxel's central projection (a*, b*), and with J the Jacobian of
// (n_o, n_z) in (a, b) every point of it lies within
//     |a - a*| <= k_a |D_m(a*, b*)| / (1 - rho),  k_a = row sum of |J^-1|,
// (likewise b) where rho bounds the relative change of D_m over the region;
// that box, a few pixels wide, holds the candidate rays.  Per candidate the
// three affine values are stepped in FP32 from the box corner (evaluated in
// FP64), so one reciprocal gives both weights.
//
// A column of voxels (i, j) decides the axes: when |g_x| > |g_y| + 1 every ray
// through the voxel's x-plane square is x-major and no y-major ray reaches the
// voxel, so only the x-plane is visited and the axis table is not read
// (likewise for y); within one voxel of the diagonal both planes are visited
// and each candidate's axis comes from the table.  The samples lie between
// the source and the pixel (0 <= g_m / D_m <= 1): when that holds with margin
// at the box corners (D_m is affine) no per-candidate test is needed,
// otherwise each candidate takes the projector's own FP64 plane-range test.
template <int M, bool AX, typename PT>
__device__ __forceinline__ float gen_plane(const PT *__restrict__ base, const uint8_t *__restrict__ axv, long ars,
                                           const ViewIdx &V, const double E[3], double gm, double go, double gz,
                                           double pm, int nu, int nv) {
    constexpr int O = 1 - M;
    const double um = V.u[M], vm = V.v[M];
    const double O0 = gm * E[O] - go * E[M], Oa = gm * V.u[O] - go * um, Ob = gm * V.v[O] - go * vm;
    const double Z0 = gm * E[2] - gz * E[M], Za = gm * V.u[2] - gz * um, Zb = gm * V.v[2] - gz * vm;
    const float fdet = (float)(Oa * Zb - Ob * Za);
    if (!(fabsf(fdet) > 0.f)) return 0.f;  // the square's image is degenerate
    const float rdet = 1.f / fdet;
    const float ac = (float)(Ob * Z0 - Zb * O0) * rdet;
    const float bc = (float)(Za * O0 - Oa * Z0) * rdet;
    const float ka = (fabsf((float)Zb) + fabsf((float)Ob)) * fabsf(rdet);
    const float kb = (fabsf((float)Za) + fabsf((float)Oa)) * fabsf(rdet);
    const float fum = (float)um, fvm = (float)vm;
    const float dc = fmaf(fvm, bc, fmaf(fum, ac, (float)E[M]));
    const float rho = fabsf(fum) * ka + fabsf(fvm) * kb;
    float wa = 1e30f, wb = 1e30f;  // the whole detector when the bound fails
    if (rho < 0.5f) {
        const float sc = fabsf(dc) / (1.f - rho);
        wa = ka * sc;
        wb = kb * sc;
    }
    // margin for the FP32 centre (relative error ~1e-7 of |a*|)
    const float ma = 2e-3f + 1e-5f * fabsf(ac), mb = 2e-3f + 1e-5f * fabsf(bc);
    const float fa0 = fmaxf(ceilf(ac - wa - ma), 0.f), fa1 = fminf(floorf(ac + wa + ma), (float)(nu - 1));
    const float fb0 = fmaxf(ceilf(bc - wb - mb), 0.f), fb1 = fminf(floorf(bc + wb + mb), (float)(nv - 1));
    if (!(fa0 <= fa1 && fb0 <= fb1)) return 0.f;  // off the detector (or NaN)
    const int a0 = (int)fa0, a1 = (int)fa1, b0 = (int)fb0, b1 = (int)fb1;
    const double da0 = a0, db0 = b0;
    const float no0 = (float)(O0 + Oa * da0 + Ob * db0);
    const float nz0 = (float)(Z0 + Za * da0 + Zb * db0);
    const float d0 = (float)(E[M] + um * da0 + vm * db0);
    const float oa = (float)Oa, ob = (float)Ob, za = (float)Za, zb = (float)Zb;
    // 0 <= g_m / D_m <= 1 over the whole box?
    const float sg = gm > 0.0 ? 1.f : -1.f, agm = fabsf((float)gm);
    const float pa = (float)(a1 - a0), pb = (float)(b1 - b0);
    const float dmin = fminf(fminf(sg * d0, sg * fmaf(pa, fum, d0)),
                             fminf(sg * fmaf(pb, fvm, d0), sg * fmaf(pb, fvm, fmaf(pa, fum, d0))));
    const bool inside = gm != 0.0 && dmin > agm * (1.f + 1e-5f) + 1e-6f;
    const double ccu = 0.5 * (nu - 1), ccv = 0.5 * (nv - 1);
    float sum = 0.f;
    for (int a = a0; a <= a1; ++a) {
        const float p = (float)(a - a0);
        const float no_r = fmaf(p, oa, no0), nz_r = fmaf(p, za, nz0), d_r = fmaf(p, fum, d0);
        const PT *col = base + (long)a * nv;
        for (int b = b0; b <= b1; ++b) {
            const float q = (float)(b - b0);
            const float r = __builtin_amdgcn_rcpf(fmaf(q, fvm, d_r));
            const float wo = 1.f - fabsf(fmaf(q, ob, no_r) * r);
            const float wz = 1.f - fabsf(fmaf(q, zb, nz_r) * r);
            bool ok = wo > 0.f && wz > 0.f;
            if (AX && ok) ok = axv[b * ars + a] == M;
            if (!inside && ok) {
                const double Dm = (V.d[M] + (a - ccu) * um + (b - ccv) * vm) - V.s[M];
                ok = pm >= fmin(V.s[M], V.s[M] + Dm) && pm <= fmax(V.s[M], V.s[M] + Dm);
            }
            if (ok) sum = fmaf(wo * wz, load_f(col, b), sum);
        }
    }
    return sum;
}

// One lane per voxel, lanes along z; per-view sums in FP32, summed in FP64.
template <typename PT>
__global__ __launch_bounds__(256) void k_backproject_gen(const PT *__restrict__ pt, float *__restrict__ vol,
                                                         float *__restrict__ part, const ViewIdx *__restrict__ views,
                                                         const uint8_t *__restrict__ axis, long axis_view_stride,
                                                         long axis_row_stride, int nx, int ny, int nz, int nu, int nv,
                                                         int nviews_sub, int view0, int view_step, int per_chunk) {
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int zchunks = (nz + 63) / 64;
    const int k = (wave % zchunks) * 64 + lane;
    const int ij = wave / zchunks;
    const int i = ij % nx, j = ij / nx;
    if (j >= ny) return;  // whole wave; no barrier below
    double acc = 0.0;
    const int vbeg = blockIdx.y * per_chunk;
    const int vend = min(nviews_sub, vbeg + per_chunk);
    for (int vl = vbeg; vl < vend && k < nz; ++vl) {
        const int v = view0 + vl * view_step;
        const ViewIdx &V = views[v];
        const double ccu = 0.5 * (nu - 1), ccv = 0.5 * (nv - 1);
        double E[3];
#pragma unroll
        for (int e = 0; e < 3; ++e) E[e] = (V.d[e] - ccu * V.u[e] - ccv * V.v[e]) - V.s[e];
        const double gx = i - V.s[0], gy = j - V.s[1], gz = k - V.s[2];
        const double ax = fabs(gx), ay = fabs(gy), tol = 1.0 + 1e-6 * (ax + ay);
        const PT *base = pt + (long)vl * nu * nv;
        const uint8_t *axv = axis + v * axis_view_stride;
        float pv;
        if (ax - ay > tol)
            pv = gen_plane<0, false>(base, axv, axis_row_stride, V, E, gx, gy, gz, (double)i, nu, nv);
        else if (ay - ax > tol)
            pv = gen_plane<1, false>(base, axv, axis_row_stride, V, E, gy, gx, gz, (double)j, nu, nv);
        else
            pv = gen_plane<0, true>(base, axv, axis_row_stride, V, E, gx, gy, gz, (double)i, nu, nv) +
                 gen_plane<1, true>(base, axv, axis_row_stride, V, E, gy, gx, gz, (double)j, nu, nv);
        acc += (double)pv;
    }
    if (k < nz) {
        const long o = ((long)k * ny + j) * nx + i;
        if (gridDim.y == 1) vol[o] = (float)acc;
        else part[(long)blockIdx.y * nx * ny * nz + o] = (float)acc;
    }
}

hipError_t launch_backproject_gen(const void *pt, int pt_dtype, float *vol, float *scratch, const Level &L, int view0,
                                  int view_step, int nviews_sub, hipStream_t s) {
    const long waves = (long)((L.nz + 63) / 64) * L.nx * L.ny;
    long c = (16384 + waves - 1) / waves;
    if (c > 64) c = 64;
    if (c > nviews_sub) c = nviews_sub;
    const int nchunks = c < 1 ? 1 : (int)c;
    if (nchunks > 1 && !scratch) return hipErrorInvalidValue;
    const int per = (nviews_sub + nchunks - 1) / nchunks;
    dim3 grid((unsigned)((waves + 3) / 4), (unsigned)nchunks);
    const long avs = L.separable ? (long)L.nu : (long)L.nu * L.nv;
    const long ars = L.axis_row_stride;
    if (pt_dtype == MGCT_F32)
        k_backproject_gen<float><<<grid, 256, 0, s>>>((const float *)pt, vol, scratch, L.d_views, L.d_axis, avs, ars,
                                                      L.nx, L.ny, L.nz, L.nu, L.nv, nviews_sub, view0, view_step,
                                                      per);
    else if (pt_dtype == MGCT_F16)
        k_backproject_gen<_Float16><<<grid, 256, 0, s>>>((const _Float16 *)pt, vol, scratch, L.d_views, L.d_axis, avs,
                                                         ars, L.nx, L.ny, L.nz, L.nu, L.nv, nviews_sub, view0,
                                                         view_step, per);
    else
        return hipErrorInvalidValue;
    if (nchunks > 1) {
        const long nvox = (long)L.nx * L.ny * L.nz;
        unsigned g = (unsigned)std::min<long>((nvox + 255) / 256, 65535L * 4);
        k_sum_chunks<float><<<g, 256, 0, s>>>(scratch, vol, nvox, nchunks);
    }
    return hipGetLastError();
}

size_t backproject_gen_scratch_bytes(const Level &L, int nviews_sub) {
    const long waves = (long)((L.nz + 63) / 64) * L.nx * L.ny;
    long c = (16384 + waves - 1) / waves;
    if (c > 64) c = 64;
    if (c > nviews_sub) c = nviews_sub;
    return c > 1 ? (size_t)c * L.vox() * sizeof(float) : 0;
}

}  // namespace mgct
