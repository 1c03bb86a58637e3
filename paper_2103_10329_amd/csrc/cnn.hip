// Learned preconditioner: a residual 3-D CNN applied to the filtered
// Landweber update u (eq. 4's step), out = u + f(u), with f four 3^3
// convolutions 1 -> 16 -> 32 -> 32 -> 1 (zero "same" padding, erf-GELU after
// the first three).  BF16 weights and activations, FP32 accumulation, FP32
// master weights and Adam state.
//
// Layout: activations channels-last [voxel][channel] (voxel = (z*ny + y)*nx
// + x).  The two 32-output layers (and their input gradients) are implicit
// GEMMs on the matrix cores: a wave computes 32 consecutive voxels along x
// times 32 output channels with v_mfma_f32_32x32x16_bf16, K running over the
// 27 taps times the input channels in chunks of 16; each lane's A operand is
// the 8 contiguous channels of one shifted voxel (one 16-byte load).  The
// weight gradients of those layers are GEMMs with K = voxels on
// channels-first copies (8 consecutive voxels per lane).  The 1-channel first
// and last layers run on the vector ALUs.
#include <hip/hip_runtime.h>
#include <math.h>

#include "mgct_internal.h"

namespace mgct {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// offsets into the FP32 master parameter vector ([co][ci][kz][ky][kx] per layer)
constexpr int kW1 = 0, kB1 = 432, kW2 = 448, kB2 = 14272, kW3 = 14304, kB3 = 41952, kW4 = 41984, kB4 = 42848;
static_assert(kB4 + 1 == kCnnParams, "parameter layout");

__device__ __forceinline__ float bf(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ uint16_t to_bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
// FP32 -> BF16 bits, round to nearest even in one conversion instruction
// (same as to_bf for every finite value)
__device__ __forceinline__ uint16_t to_bf_cvt(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

// Two FP32 values -> two BF16 (round to nearest even) packed low, high, in
// one conversion instruction.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((floatx2){lo, hi}, bf16x2));
}

// GELU x Phi(x) for the forward activations, without branches, written as
// max(x, 0) - |x| erfc(y) / 2 with y = |x| / sqrt(2) (equal to x Phi(x) for
// either sign), erfc(y) = (a1 t + ... + a5 t^5) exp(-y^2), t = 1 / (1 + p y):
// the rational approximation of Abramowitz & Stegun, Handbook of
// Mathematical Functions, 7.1.26 (|error| <= 1.5e-7 on erf), its
// coefficients halved (exactly) to give erfc(y) / 2; exp(-x^2 / 2) as
// exp2(-x^2 / (2 ln 2)); max(x, 0) as an integer maximum of the bit pattern
// (a float with the sign bit set is a negative integer).  The result is
// stored in BF16 (relative step 2^-8), so the difference to the exact erf
// shows only as a rare rounding flip (the coarser 7.1.28, one reciprocal and
// no exponential, measurably raised the flips in the negative tail, where
// GELU is small and its relative error large); the backward pass keeps the
// exact derivative.  Finite inputs.
__device__ __forceinline__ float gelu(float x) {
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f * 0.70710678118654752f, ax, 1.f));
    float q = fmaf(0.5f * 1.061405429f, t, 0.5f * -1.453152027f);
    q = fmaf(q, t, 0.5f * 1.421413741f);
    q = fmaf(q, t, 0.5f * -0.284496736f);
    q = fmaf(q, t, 0.5f * 0.254829592f);
    q *= t * __builtin_amdgcn_exp2f(-0.72134752044448170f * x * x);  // erfc(y) / 2
    return fmaf(-ax, q, __int_as_float(max(__float_as_int(x), 0)));
}
__device__ __forceinline__ float gelu_grad(float x) {
    return 0.5f * (1.f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

struct Dims {
    int nx, ny, nz;
};
__device__ __forceinline__ bool tap_voxel(const Dims &d, int x, int y, int z, int t, long &v) {
    const int xx = x + (t % 3) - 1, yy = y + (t / 3) % 3 - 1, zz = z + t / 9 - 1;
    if (xx < 0 || yy < 0 || zz < 0 || xx >= d.nx || yy >= d.ny || zz >= d.nz) return false;
    v = ((long)zz * d.ny + yy) * d.nx + xx;
    return true;
}

// ------------------------------------------------------------ weights ----

// P2f[t][co][ci] (ci<16), P3f[t][co][ci], P3d[t][ci][co] = W3[co][ci][26-t],
// P2d[t][ci][co] = W2[co][ci][26-t] for ci < 16, zero for ci in 16..31.
__global__ void k_pack_weights(const float *__restrict__ w, uint16_t *P2f, uint16_t *P3f, uint16_t *P3d,
                               uint16_t *P2d) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 27 * 32 * 16) {
        const int t = i / 512, co = (i / 16) % 32, ci = i % 16;
        P2f[i] = to_bf(w[kW2 + (co * 16 + ci) * 27 + t]);
    }
    if (i < 27 * 32 * 32) {
        const int t = i / 1024, a = (i / 32) % 32, c = i % 32;
        P3f[i] = to_bf(w[kW3 + (a * 32 + c) * 27 + t]);          // a = co, c = ci
        P3d[i] = to_bf(w[kW3 + (c * 32 + a) * 27 + (26 - t)]);   // a = ci, c = co
        P2d[i] = a < 16 ? to_bf(w[kW2 + (c * 16 + a) * 27 + (26 - t)]) : (uint16_t)0;
    }
}

// Layer 4 on the matrix cores (k_conv4_ym): P4[hl][dz][kc][j][16] holds, for
// slot j = (dx, dy) (j = 3 (dy + 1) + dx + 1 < 9; zero for j >= 9), input
// channels kc*16 .. kc*16 + 15 of W4[ci][tap (dx, dy, dz)] split into a BF16
// high part (hl = 0) and the BF16 rounding of the remainder (hl = 1): the two
// products together carry 16 bits of each FP32 weight.
__global__ void k_pack_weights4(const float *__restrict__ w, uint16_t *P4) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * 3 * 2 * 32 * 16) return;
    const int hl = i / 3072, dz = (i / 1024) % 3, kc = (i / 512) % 2, j = (i / 16) % 32, ci = kc * 16 + i % 16;
    uint16_t r = 0;
    if (j < 9) {
        const int t = dz * 9 + (j / 3) * 3 + j % 3;  // kz*9 + ky*3 + kx
        const float x = w[kW4 + ci * 27 + t];
        const uint16_t hi = to_bf(x);
        r = hl ? to_bf(x - bf(hi)) : hi;
    }
    P4[i] = r;
}

// P1[p][c][k]: the three BF16 pieces (p = 0, 1, 2: top, middle and low 8 bits
// of the significand, by truncation, so that w = sum of the pieces exactly)
// of W1[c][tap k] for k < 27, zero for k = 27..31 (the MFMA's K of 32).
__device__ __forceinline__ void split_bf16x3(float x, float &p0, float &p1, float &p2) {
    p0 = __uint_as_float(__float_as_uint(x) & 0xffff0000u);
    const float r = x - p0;  // exact
    p1 = __uint_as_float(__float_as_uint(r) & 0xffff0000u);
    p2 = r - p1;  // exact, at most 8 significant bits
}
__global__ void k_pack_weights1(const float *__restrict__ w, uint16_t *P1) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * 16 * 32) return;
    const int p = i / 512, c = (i / 32) % 16, k = i % 32;
    float q[3] = {0.f, 0.f, 0.f};
    if (k < 27) split_bf16x3(w[kW1 + c * 27 + k], q[0], q[1], q[2]);
    P1[i] = (uint16_t)(__float_as_uint(q[p]) >> 16);
}

// the input with a zero border of one voxel: up[(z+1)][(y+1)][(x+1)] =
// u[z][y][x]; one block per padded row (zp, yp)
__global__ __launch_bounds__(256) void k_pad_input(const float *__restrict__ u, float *__restrict__ up, Dims d) {
    const int PX = d.nx + 2, PY = d.ny + 2;
    const int yp = blockIdx.x % PY, zp = blockIdx.x / PY;
    const bool rin = yp >= 1 && yp <= d.ny && zp >= 1 && zp <= d.nz;  // block-uniform
    const float *srow = rin ? u + ((long)(zp - 1) * d.ny + (yp - 1)) * d.nx - 1 : u;
    float *drow = up + (long)blockIdx.x * PX;
    for (int xp = threadIdx.x; xp < PX; xp += blockDim.x)
        drow[xp] = rin && xp >= 1 && xp <= d.nx ? srow[xp] : 0.f;
}

// Layer 1 (1 -> 16 channels) on the matrix cores.  A wave takes one row of
// voxels along x, 16 at a time, and computes per group D[c][x] = b1[c] +
// sum over the taps t of W1[c][t] U[t][x] as 16x16x32 MFMAs (K: the 27 taps
// and 5 zero weights).  The FP32 operands are split exactly into three BF16
// pieces (split_bf16x3), and the six piece products of combined order <= 2
// are accumulated in FP32: the three left out are below 2^-24 of the terms,
// so the sums keep FP32 accuracy.  The taps read the zero-bordered copy of
// u, none needs a bounds check; the next group's taps load while the
// current one is worked on.  Lane (n, kg) = (lane mod 16, lane / 16) holds
// row n of the weight fragments (channel n, taps 8 kg .. 8 kg + 7), column n
// of the input fragments (voxel x + n, the same taps) and of the result the
// channels 4 kg .. 4 kg + 3 of voxel x + n.
__global__ __launch_bounds__(256) void k_conv1_mfma(const float *__restrict__ up, const uint16_t *__restrict__ P1,
                                                    const float *__restrict__ w, float *__restrict__ z1,
                                                    uint16_t *__restrict__ h1, Dims d) {
    const long row = blockIdx.x * 4L + (threadIdx.x >> 6);  // z ny + y
    if (row >= (long)d.ny * d.nz) return;                      // whole wave; no barrier in this kernel
    const int lane = threadIdx.x & 63, n = lane & 15, kg = lane >> 4;
    const int y = (int)(row % d.ny), z = (int)(row / d.ny);
    const int PX = d.nx + 2, PYX = (d.ny + 2) * PX;
    bf16x8 W[3];
#pragma unroll
    for (int p = 0; p < 3; ++p) W[p] = *reinterpret_cast<const bf16x8 *>(P1 + (p * 16 + n) * 32 + kg * 8);
    floatx4 bc;
#pragma unroll
    for (int r = 0; r < 4; ++r) bc[r] = w[kB1 + 4 * kg + r];
    // tap t = 9 kz + 3 ky + kx (t / 9 and r / 3 by multiply and shift, exact
    // for t < 32) reads up at the voxel's padded base + kz PYX + ky PX + kx;
    // the zero-weight slots 27..31 read the base itself
    int off[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const int t = kg * 8 + s, kz = (t * 57) >> 9, r = t - 9 * kz, ky = (r * 11) >> 5, kx = r - 3 * ky;
        off[s] = t < 27 ? kz * PYX + ky * PX + kx : 0;
    }
    const float *src = up + ((long)z * (d.ny + 2) + y) * PX + n;
    uint2 *dst = reinterpret_cast<uint2 *>(h1 + (row * d.nx + n) * 16 + 4 * kg);
    floatx4 *zdst = z1 ? reinterpret_cast<floatx4 *>(z1 + (row * d.nx + n) * 16 + 4 * kg) : nullptr;
    float uu[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) uu[s] = src[off[s]];
    for (int x = 0; x < d.nx; x += 16) {
        uint32_t b[3][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float a0, a1, a2, c0, c1, c2;
            split_bf16x3(uu[2 * j], a0, a1, a2);
            split_bf16x3(uu[2 * j + 1], c0, c1, c2);
            // the upper halves of the two pieces, slot 2j low
            b[0][j] = __builtin_amdgcn_perm(__float_as_uint(c0), __float_as_uint(a0), 0x07060302u);
            b[1][j] = __builtin_amdgcn_perm(__float_as_uint(c1), __float_as_uint(a1), 0x07060302u);
            b[2][j] = __builtin_amdgcn_perm(__float_as_uint(c2), __float_as_uint(a2), 0x07060302u);
        }
        if (x + 16 < d.nx) {
#pragma unroll
            for (int s = 0; s < 8; ++s) uu[s] = src[x + 16 + off[s]];
        }
        bf16x8 B[3];
#pragma unroll
        for (int p = 0; p < 3; ++p) B[p] = __builtin_bit_cast(bf16x8, make_uint4(b[p][0], b[p][1], b[p][2], b[p][3]));
        // smallest products first
        floatx4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W[2], B[0], bc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W[1], B[1], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W[0], B[2], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W[1], B[0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W[0], B[1], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W[0], B[0], acc, 0, 0, 0);
        if (zdst) zdst[x * 4] = acc;
        dst[x * 4] = make_uint2(pack_bf16x2(gelu(acc[0]), gelu(acc[1])), pack_bf16x2(gelu(acc[2]), gelu(acc[3])));
    }
}

// ------------------------------------------------------ VALU layers ----

// out[v] = u[v] + b4 + sum_{t, ci} W4[ci][t] h3[v + off_t][ci]
__global__ __launch_bounds__(256) void k_conv4_fwd(const uint16_t *__restrict__ h3, const float *__restrict__ w,
                                                   const float *__restrict__ u, float *__restrict__ out, Dims d) {
    const long n = (long)d.nx * d.ny * d.nz;
    const long v = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (v >= n) return;
    int x, y, z;
    split3(v, d.nx, d.ny, x, y, z);
    float acc = w[kB4];
    for (int t = 0; t < 27; ++t) {
        long q;
        if (!tap_voxel(d, x, y, z, t, q)) continue;
        const uint4 *p = reinterpret_cast<const uint4 *>(h3 + q * 32);
#pragma unroll
        for (int c4 = 0; c4 < 4; ++c4) {
            const uint4 r = p[c4];
            const uint32_t wd[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int ci = c4 * 8 + e * 2;
                acc = fmaf(w[kW4 + ci * 27 + t], __uint_as_float(wd[e] << 16), acc);
                acc = fmaf(w[kW4 + (ci + 1) * 27 + t], __uint_as_float(wd[e] & 0xffff0000u), acc);
            }
        }
    }
    out[v] = u[v] + acc;
}

// loss partials and dout = 2 (out - target) / n
__global__ __launch_bounds__(256) void k_mse(const float *__restrict__ out, const float *__restrict__ target,
                                             float *__restrict__ dout, double *__restrict__ partials, long n) {
    double acc = 0.0;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const float e = out[i] - target[i];
        dout[i] = 2.f * e / (float)n;
        acc += (double)e * e;
    }
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// dz3[v][ci] = GELU'(z3[v][ci]) * sum_t W4[ci][t] dout[v - off_t]
__global__ __launch_bounds__(256) void k_conv4_bwd_input(const float *__restrict__ dout, const float *__restrict__ w,
                                                         const float *__restrict__ z3, uint16_t *__restrict__ dz3,
                                                         Dims d) {
    // a block covers 256 consecutive voxels; their z3 rows are read and
    // their dz3 rows written through LDS, so the global accesses are
    // contiguous (one thread per voxel would touch 64 rows per access)
    __shared__ float zs[256 * 33];
    const long n = (long)d.nx * d.ny * d.nz;
    const long vb = blockIdx.x * 256L;
    for (int e = threadIdx.x; e < 256 * 32; e += 256)
        zs[(e >> 5) * 33 + (e & 31)] = vb + (e >> 5) < n ? z3[vb * 32 + e] : 0.f;
    __syncthreads();
    const long v = vb + threadIdx.x;
    float o[32];
    if (v < n) {
        int x, y, z;
        split3(v, d.nx, d.ny, x, y, z);
        float g[27];
#pragma unroll
        for (int t = 0; t < 27; ++t) {
            long q;
            g[t] = tap_voxel(d, x, y, z, 26 - t, q) ? dout[q] : 0.f;  // v - off_t = v + off_(26-t)
        }
#pragma unroll
        for (int ci = 0; ci < 32; ++ci) {
            float acc = 0.f;
#pragma unroll
            for (int t = 0; t < 27; ++t) acc = fmaf(w[kW4 + ci * 27 + t], g[t], acc);
            o[ci] = acc * gelu_grad(zs[threadIdx.x * 33 + ci]);
        }
    } else {
#pragma unroll
        for (int ci = 0; ci < 32; ++ci) o[ci] = 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int ci = 0; ci < 32; ++ci) zs[threadIdx.x * 33 + ci] = o[ci];
    __syncthreads();
    for (int e = threadIdx.x; e < 256 * 32; e += 256)
        if (vb + (e >> 5) < n) dz3[vb * 32 + e] = to_bf(zs[(e >> 5) * 33 + (e & 31)]);
}

// Weight gradient of a layer with one input channel (layer 1: X = u FP32,
// G = dz1 [v][16] BF16) or one output channel (layer 4: X = h3 [v][32] BF16,
// G = dout FP32): grad[o] = sum_v X(v + off_t(o), c(o)) * G(v, c'(o)), plus
// the bias gradients (sum_v G) in the last slots.  A block covers one 32-wide
// x tile of `rpc` consecutive rows (y, z); per row it stages the 3 x 3
// neighbouring rows of X (34 wide, zero outside the volume) and the row of G
// in LDS, and each thread accumulates up to four parameters.
// partial[block][R], block = rowchunk * (nx / 32) + xtile.  nx % 32 == 0.
template <int MODE>  // 1: layer 1 (R = 16*27 + 16), 4: layer 4 (R = 32*27 + 1)
__global__ __launch_bounds__(256) void k_wgrad_valu(const float *__restrict__ xf, const uint16_t *__restrict__ xh,
                                                    const uint16_t *__restrict__ gh, const float *__restrict__ gf,
                                                    float *__restrict__ partial, Dims d, int rpc) {
    constexpr int R = MODE == 1 ? 16 * 27 + 16 : 32 * 27 + 1;
    constexpr int C = MODE == 1 ? 1 : 32;    // channels of X
    constexpr int CG = MODE == 1 ? 16 : 1;   // channels of G
    constexpr int CS = MODE == 1 ? 1 : 33;   // LDS stride per x (one pad float against bank conflicts)
    constexpr int NP = (R + 255) / 256;
    __shared__ float xs[9][34 * CS];
    __shared__ float gs[32 * CG];
    const int nxt = d.nx / 32;
    const int xt = blockIdx.x % nxt, rc = blockIdx.x / nxt;
    const int x0 = xt * 32;
    const int nrows = d.ny * d.nz;
    const int r0 = rc * rpc, r1 = min(nrows, r0 + rpc);
    float acc[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) acc[p] = 0.f;
    for (int row = r0; row < r1; ++row) {
        const int y = row % d.ny, z = row / d.ny;
        __syncthreads();  // previous row's reads are done
        if (MODE == 1) {
            for (int e = threadIdx.x; e < 9 * 34; e += 256) {
                const int tr = e / 34, xl = e % 34;
                const int yy = y + tr % 3 - 1, zz = z + tr / 3 - 1, xx = x0 + xl - 1;
                float val = 0.f;
                if (yy >= 0 && yy < d.ny && zz >= 0 && zz < d.nz && xx >= 0 && xx < d.nx)
                    val = xf[((long)zz * d.ny + yy) * d.nx + xx];
                xs[tr][xl] = val;
            }
        } else {
            // eight channels (16 bytes) per load
            for (int e = threadIdx.x; e < 9 * 34 * 4; e += 256) {
                const int tr = e / (34 * 4), rem = e % (34 * 4);
                const int xl = rem >> 2, c8 = (rem & 3) * 8;
                const int yy = y + tr % 3 - 1, zz = z + tr / 3 - 1, xx = x0 + xl - 1;
                uint16_t h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                if (yy >= 0 && yy < d.ny && zz >= 0 && zz < d.nz && xx >= 0 && xx < d.nx) {
                    const long q = ((long)zz * d.ny + yy) * d.nx + xx;
                    __builtin_memcpy(h, __builtin_assume_aligned(xh + q * 32 + c8, 16), 16);
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) xs[tr][xl * CS + c8 + k] = bf(h[k]);
            }
        }
        const long gv = (long)row * d.nx + x0;
        for (int e = threadIdx.x; e < 32 * CG; e += 256)
            gs[e] = MODE == 1 ? bf(gh[gv * 16 + e]) : gf[gv + e];
        __syncthreads();
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int o = threadIdx.x + 256 * p;
            if (o >= R) continue;
            float a = acc[p];
            if (o < 27 * (MODE == 1 ? 16 : 32)) {
                const int c2 = o / 27, t = o % 27;  // layer 1: c2 = co (of G); layer 4: c2 = ci (of X)
                const int tr = t / 3, dx = t % 3;   // tr = 3 (dz + 1) + (dy + 1); LDS column x + dx
                if (MODE == 1) {
                    for (int x = 0; x < 32; ++x) a = fmaf(xs[tr][x + dx], gs[x * 16 + c2], a);
                } else {
                    for (int x = 0; x < 32; ++x) a = fmaf(xs[tr][(x + dx) * CS + c2], gs[x], a);
                }
            } else {
                const int c2 = o - 27 * (MODE == 1 ? 16 : 32);
                for (int x = 0; x < 32; ++x) a += gs[x * CG + c2];
            }
            acc[p] = a;
        }
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int o = threadIdx.x + 256 * p;
        if (o < R) partial[blockIdx.x * (long)R + o] = acc[p];
    }
}

// out[j] = sum_b partial[b][j] over nparts rows of R values, one wave per j:
// lane l adds rows l, l + 64, ... in FP64, then a fixed xor-shuffle tree
// (the order is fixed, so the result does not depend on scheduling).
__global__ __launch_bounds__(256) void k_sum_partials(const float *__restrict__ partial, int nparts, int R,
                                                      float *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= R) return;  // whole wave
    double acc = 0.0;
    for (int b = lane; b < nparts; b += 64) acc += (double)partial[(long)b * R + j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) out[j] = (float)acc;
}

// ------------------------------------------------------ matrix cores ----

// MODE 0 (forward): out channels 32, z = acc + bias -> zout (FP32, may be
//   null), hout = BF16 GELU(z).
// MODE 1 (input gradient): out channels NOUT (16 or 32), hout = BF16
//   acc * GELU'(zprev).
// X: [v][CI] BF16; P: [27][32][CI] BF16 (B operand, n-major).  nx % 32 == 0.
#ifndef MGCT_CONV_ROWS
#define MGCT_CONV_ROWS 2
#endif
// Output rows (y) per wave: each weight fragment is loaded once per tap and
// channel chunk and used for all of them.
constexpr int kConvRows = MGCT_CONV_ROWS;

template <int CI, int MODE>
__global__ __launch_bounds__(256) void k_conv_mfma(const uint16_t *__restrict__ X, const uint16_t *__restrict__ P,
                                                   const float *__restrict__ bias, const float *__restrict__ zprev,
                                                   float *__restrict__ zout, uint16_t *__restrict__ hout, int nout,
                                                   Dims d) {
    constexpr int NT = kConvRows;
    const int lane = threadIdx.x & 63;
    const long wave = blockIdx.x * 4L + (threadIdx.x >> 6);
    const int nxt = d.nx / 32, nyt = (d.ny + NT - 1) / NT;
    if (wave >= (long)nxt * nyt * d.nz) return;  // whole wave; no barrier below
    int xt, yt, z;
    split3(wave, nxt, nyt, xt, yt, z);
    const int x0 = xt * 32, y0 = yt * NT;
    const int m = lane & 31, kh = lane >> 5;
    floatx16 acc[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) acc[i] = floatx16{};
    for (int t = 0; t < 27; ++t) {
        long q[NT];
        bool ok[NT];
#pragma unroll
        for (int i = 0; i < NT; ++i) {
            q[i] = 0;
            ok[i] = y0 + i < d.ny && tap_voxel(d, x0 + m, y0 + i, z, t, q[i]);
        }
#pragma unroll
        for (int kc = 0; kc < CI / 16; ++kc) {
            const bf16x8 b = *reinterpret_cast<const bf16x8 *>(P + ((long)t * 32 + m) * CI + kc * 16 + kh * 8);
#pragma unroll
            for (int i = 0; i < NT; ++i) {
                bf16x8 a = {};
                if (ok[i]) a = *reinterpret_cast<const bf16x8 *>(X + q[i] * CI + kc * 16 + kh * 8);
                acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[i], 0, 0, 0);
            }
        }
    }
    // D[i][j]: column j = lane % 32, row i = 8 (r / 4) + 4 (lane / 32) + r % 4 for register r
    const int col = m;
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        if (y0 + i >= d.ny) break;  // wave-uniform
        const long v0 = ((long)z * d.ny + y0 + i) * d.nx + x0;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = 8 * (r >> 2) + 4 * kh + (r & 3);
            const long v = v0 + row;
            if (MODE == 0) {
                const float zv = acc[i][r] + bias[col];
                if (zout) zout[v * 32 + col] = zv;
                hout[v * 32 + col] = to_bf(gelu(zv));
            } else if (col < nout) {
                hout[v * nout + col] = to_bf(acc[i][r] * gelu_grad(zprev[v * nout + col]));
            }
        }
    }
}

// The same convolution with the input staged in LDS: a block covers one
// 32-voxel x tile, 4 * kConvLdsRows rows (y) and one z; it loads the 3 x (rows+2)
// x 34 voxel neighbourhood once (16-byte loads along the contiguous
// channels-last rows, zero outside the volume) and each wave reads its A
// fragments from there, so an input value is fetched from memory about four
// times instead of once per tap.  Voxels are padded to CI + 8 channels
// against LDS bank conflicts.  Same operands and order as k_conv_mfma.
#ifndef MGCT_CONV_LDS_ROWS
#define MGCT_CONV_LDS_ROWS 2
#endif
constexpr int kConvLdsRows = MGCT_CONV_LDS_ROWS;  // output rows per wave of the LDS-staged kernel

template <int CI, int MODE>
__global__ __launch_bounds__(256) void k_conv_mfma_lds(const uint16_t *__restrict__ X,
                                                       const uint16_t *__restrict__ P,
                                                       const float *__restrict__ bias,
                                                       const float *__restrict__ zprev, float *__restrict__ zout,
                                                       uint16_t *__restrict__ hout, int nout, Dims d) {
    constexpr int NT = kConvLdsRows, YB = 4 * NT, SY = YB + 2, CP = CI + 8;
    extern __shared__ uint16_t xs[];  // [3][SY][34][CP]
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nxt = d.nx / 32, nyb = (d.ny + YB - 1) / YB;
    int xt, yb, z;
    split3(blockIdx.x, nxt, nyb, xt, yb, z);
    const int x0 = xt * 32, y0 = yb * YB;
    // stage: (zz, yy, xx) voxels of CI channels as CI / 8 chunks of 16 bytes
    constexpr int CH = CI / 8, NV = 3 * SY * 34;
    for (int e = threadIdx.x; e < NV * CH; e += 256) {
        const int vox = e / CH, c8 = (e % CH) * 8;
        const int lx = vox % 34, ly = (vox / 34) % SY, lz = vox / (34 * SY);
        const int xx = x0 + lx - 1, yy = y0 + ly - 1, zz = z + lz - 1;
        uint4 val = {0u, 0u, 0u, 0u};
        if (xx >= 0 && xx < d.nx && yy >= 0 && yy < d.ny && zz >= 0 && zz < d.nz)
            val = *reinterpret_cast<const uint4 *>(X + (((long)zz * d.ny + yy) * d.nx + xx) * CI + c8);
        *reinterpret_cast<uint4 *>(xs + vox * CP + c8) = val;
    }
    __syncthreads();
    const int m = lane & 31, kh = lane >> 5;
    const int r0 = w * NT;  // the wave's first row within the block
    floatx16 acc[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) acc[i] = floatx16{};
    for (int t = 0; t < 27; ++t) {
        const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
#pragma unroll
        for (int kc = 0; kc < CI / 16; ++kc) {
            const bf16x8 b = *reinterpret_cast<const bf16x8 *>(P + ((long)t * 32 + m) * CI + kc * 16 + kh * 8);
#pragma unroll
            for (int i = 0; i < NT; ++i) {
                const int vox = ((1 + dz) * SY + (r0 + i + 1 + dy)) * 34 + (m + 1 + dx);
                const bf16x8 a = *reinterpret_cast<const bf16x8 *>(xs + vox * CP + kc * 16 + kh * 8);
                acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[i], 0, 0, 0);
            }
        }
    }
    const int col = m;
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        const int y = y0 + r0 + i;
        if (y >= d.ny) break;  // wave-uniform
        const long v0 = ((long)z * d.ny + y) * d.nx + x0;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = 8 * (r >> 2) + 4 * kh + (r & 3);
            const long v = v0 + row;
            if (MODE == 0) {
                const float zv = acc[i][r] + bias[col];
                if (zout) zout[v * 32 + col] = zv;
                hout[v * 32 + col] = to_bf(gelu(zv));
            } else if (col < nout) {
                hout[v * nout + col] = to_bf(acc[i][r] * gelu_grad(zprev[v * nout + col]));
            }
        }
    }
}

// Forward convolution of the two 32-output layers on large grids:
// persistent and weight-stationary.  A wave holds all 27 x CI/16 weight
// fragments of the layer (the B operands) in registers, loaded once, and
// owns one 32-voxel x tile at one z at a time, marching up y: the A fragment
// of an input row at one (dx, dz) shift and channel chunk serves the three
// output rows it reaches (dy = -1, 0, 1), whose accumulators rotate as the
// march goes on, so every input fragment is loaded once for three MFMAs.
// A block's 4 waves take 4 consecutive z (their input rows overlap in the
// vector cache) and blocks loop over (x tile, z quad) items.  The products
// are those of k_conv_mfma; per output the taps are summed grouped by input
// row (dy, then dz, dx) rather than in tap order, so results agree to FP32
// rounding.  nx % 32 == 0.
template <int CI> struct ConvW {
    bf16x8 f[27][CI / 16];
};
// One dz slice of an input row's A fragments: [dx][channel chunk].
template <int CI> struct ConvSlice {
    bf16x8 a[3][CI / 16];
};

// 32 zero channels: lanes whose shifted voxel lies outside the volume read
// their A fragment from here (the address is chosen before the load, so no
// select waits for it).
__device__ const uint16_t kConvZeros[32] = {};

// slice dz (0..2 for z - 1 .. z + 1) of input row yi
template <int CI>
__device__ __forceinline__ void conv_ym_load(ConvSlice<CI> &S, const uint16_t *__restrict__ X, const Dims &d,
                                             int x0, int z, int yi, int dz, int m, int kh) {
    const int zz = z + dz - 1;
    const bool zok = yi >= 0 && yi < d.ny && zz >= 0 && zz < d.nz;
    const long rowbase = zok ? ((long)zz * d.ny + yi) * d.nx : 0;
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
        const int xx = x0 + m + dx - 1;
        const bool ok = zok && xx >= 0 && xx < d.nx;
        const uint16_t *src = (ok ? X + (rowbase + xx) * CI : kConvZeros) + kh * 8;
#pragma unroll
        for (int kc = 0; kc < CI / 16; ++kc)
            S.a[dx][kc] = *reinterpret_cast<const bf16x8 *>(src + (ok ? kc * 16 : 0));
    }
}

// aP: output row yi - 1 (tap dy = +1), a0: yi (dy = 0), aN: yi + 1 (dy = -1)
template <int CI, int DZ>
__device__ __forceinline__ void conv_ym_mfma(const ConvSlice<CI> &S, const ConvW<CI> &W, floatx16 &aP,
                                             floatx16 &a0, floatx16 &aN) {
#pragma unroll
    for (int dx = 0; dx < 3; ++dx)
#pragma unroll
        for (int kc = 0; kc < CI / 16; ++kc) {
            const int tb = DZ * 9 + dx;
            aN = __builtin_amdgcn_mfma_f32_32x32x16_bf16(S.a[dx][kc], W.f[tb][kc], aN, 0, 0, 0);
            a0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(S.a[dx][kc], W.f[tb + 3][kc], a0, 0, 0, 0);
            aP = __builtin_amdgcn_mfma_f32_32x32x16_bf16(S.a[dx][kc], W.f[tb + 6][kc], aP, 0, 0, 0);
        }
}

// output row yo of the wave's tile: bias bc (this lane's channel), GELU, BF16
// (and the FP32 pre-activation)
__device__ __forceinline__ void conv_ym_store(floatx16 &acc, float bc, float *zout, uint16_t *__restrict__ hout,
                                              const Dims &d, int x0, int yo, int z, int m, int kh) {
    if (yo >= 0 && yo < d.ny) {
        const long v0 = ((long)z * d.ny + yo) * d.nx + x0;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const long v = v0 + 8 * (r >> 2) + 4 * kh + (r & 3);
            const float zv = acc[r] + bc;
            if (zout) zout[v * 32 + m] = zv;
            hout[v * 32 + m] = to_bf(gelu(zv));
        }
    }
    acc = floatx16{};
}

// One input row: its three slices from buffers 0, 1, 2 (slices 0 and 1
// already loaded on entry), the loads running two slices ahead (on exit
// buffers 0 and 1 hold the next row's slices 0 and 1), then the completed
// output row yi - 1.
template <int CI>
__device__ __forceinline__ void conv_ym_step(ConvSlice<CI> (&B)[3], const uint16_t *__restrict__ X,
                                             const ConvW<CI> &W, const Dims &d, int x0, int z, int yi, int m,
                                             int kh, floatx16 &aP, floatx16 &a0, floatx16 &aN, float bc,
                                             float *zout, uint16_t *__restrict__ hout) {
    conv_ym_load<CI>(B[2], X, d, x0, z, yi, 2, m, kh);
    conv_ym_mfma<CI, 0>(B[0], W, aP, a0, aN);
    conv_ym_load<CI>(B[0], X, d, x0, z, yi + 1, 0, m, kh);
    conv_ym_mfma<CI, 1>(B[1], W, aP, a0, aN);
    conv_ym_load<CI>(B[1], X, d, x0, z, yi + 1, 1, m, kh);
    conv_ym_mfma<CI, 2>(B[2], W, aP, a0, aN);
    conv_ym_store(aP, bc, zout, hout, d, x0, yi - 1, z, m, kh);
}

template <int CI>
__global__ __launch_bounds__(256, 1) void k_conv_ym(const uint16_t *__restrict__ X, const uint16_t *__restrict__ P,
                                                    const float *__restrict__ bias, float *__restrict__ zout,
                                                    uint16_t *__restrict__ hout, Dims d, int n_items) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m = lane & 31, kh = lane >> 5;
    ConvW<CI> W;
#pragma unroll
    for (int t = 0; t < 27; ++t)
#pragma unroll
        for (int kc = 0; kc < CI / 16; ++kc)
            W.f[t][kc] = *reinterpret_cast<const bf16x8 *>(P + ((long)t * 32 + m) * CI + kc * 16 + kh * 8);
    const int nxt = d.nx / 32;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int x0 = (it % nxt) * 32, z = (it / nxt) * 4 + w;
        if (z >= d.nz) continue;  // whole wave; no barrier in this kernel
        // input rows -1 .. ny (row yi completes output row yi - 1); the
        // three accumulators rotate, three rows per trip
        const float bc = bias[m];
        floatx16 A0{}, A1{}, A2{};
        ConvSlice<CI> B[3];
        conv_ym_load<CI>(B[0], X, d, x0, z, -1, 0, m, kh);
        conv_ym_load<CI>(B[1], X, d, x0, z, -1, 1, m, kh);
        for (int yi = -1; yi <= d.ny; yi += 3) {
            conv_ym_step<CI>(B, X, W, d, x0, z, yi, m, kh, A0, A1, A2, bc, zout, hout);
            if (yi + 1 > d.ny) break;
            conv_ym_step<CI>(B, X, W, d, x0, z, yi + 1, m, kh, A1, A2, A0, bc, zout, hout);
            if (yi + 2 > d.ny) break;
            conv_ym_step<CI>(B, X, W, d, x0, z, yi + 2, m, kh, A2, A0, A1, bc, zout, hout);
        }
    }
}

// The same layers with the input rows staged in LDS by the data mover: a
// block's 4 waves (4 consecutive z) share a ring of kConvRing input rows
// (the 6 z rows z0 - 1 .. z0 + 4 times the 34 x of the tile and its two
// neighbours, every channel), filled by global-to-LDS loads three rows ahead
// of the row being worked on, so that the latency of memory is covered by
// three rows of MFMAs instead of two dz slices.  Each wave issues the same
// number of 16-byte transfers per row (positions past the row's data fill
// the slot's padding from the zero array), waits for its own transfers of
// the row it is about to read (the row's transfers were issued before the
// later rows', and loads complete in order), then all waves meet at a
// barrier.  The 16-byte chunks of a voxel are laid out (conv_slot) so that
// a fragment read (16 lanes, consecutive x, one chunk each) touches 16
// different groups of banks.  Accumulator of output row o: A[o mod 4].
constexpr int kConvRing = 4;
#ifndef MGCT_CONV16_BLOCKS
#define MGCT_CONV16_BLOCKS 2
#endif
#ifndef MGCT_CONV32_PAD
#define MGCT_CONV32_PAD 0
#endif
template <int CI, int NW = 4, int XW = 34> struct ConvLds {
    static constexpr int C = CI / 8;                                  // 16-byte chunks per voxel
    static constexpr int CP = CI == 32 && MGCT_CONV32_PAD ? C + 1 : C;  // chunk slots per voxel in LDS
    static constexpr int X = XW;                                      // staged voxels per z row
    static constexpr int P = 6 * XW * CP;                             // chunk slots of one staged row
    static constexpr int L = (P + 64 * NW - 1) / (64 * NW);           // transfers per wave per row (NW waves)
    static constexpr int SLOT = L * 64 * NW;                          // chunks per ring slot (padded)
};
// LDS chunk slot of channel chunk q of voxel xi in a staged z row: the
// chunks of a voxel are permuted by an XOR with bits of xi (its own
// inverse), chosen with the LDS bank-conflict counter so that the fragment
// reads (every dx, row and voxel half) run at the conflict-free rate: for
// the 32-voxel fragments (lane = voxel + 32 chunk-of-pair) bits 2-3 of xi
// with 32 channels, bit 3 with 16; for the 16-voxel fragments of the
// eight-wave kernel (lane = voxel + 16 chunk) bits 1-2 (bits 2-3 there
// double the read time).
template <int CI, int NW = 4> __device__ __forceinline__ int conv_perm(int xi, int q) {
    if (CI == 16) return q ^ ((xi >> 3) & 1);
    if (NW == 8) return q ^ ((xi >> 1) & 3);
    return MGCT_CONV32_PAD ? q : q ^ ((xi >> 2) & 3);
}
template <int CI, int NW = 4> __device__ __forceinline__ int conv_slot(int xi, int q) {
    return xi * ConvLds<CI, NW>::CP + conv_perm<CI, NW>(xi, q);
}

// wait until at most n vector-memory operations of this wave are outstanding
template <int N> __device__ __forceinline__ void wait_vm() {
    static_assert(N < 64, "vmcnt field");
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

#ifndef MGCT_CONV_WAIT_STORES
#define MGCT_CONV_WAIT_STORES 1
#endif
constexpr int vm_cap(int n) { return n < 63 ? n : 63; }
// Wait before input row yi of the ring is read.  Its L transfers per wave
// were issued three steps earlier (or before the first step); issued after
// them are the two later rows' transfers and the output stores of the three
// steps in between (S per step; a step stores from yi = 2 on, and only in a
// wave whose z lies in the grid).  Vector-memory operations of a wave are
// counted off in issue order, so leaving that many outstanding waits for the
// row's own transfers and not for the stores behind them.
template <int L, int S> __device__ __forceinline__ void conv_row_wait(int yi, bool live) {
#if MGCT_CONV_WAIT_STORES
    const int ns = live ? (yi < 2 ? 0 : yi > 5 ? 3 : yi - 2) : 0;  // wave-uniform
    if (ns == 3)
        wait_vm<vm_cap(2 * L + 3 * S)>();
    else if (ns == 2)
        wait_vm<vm_cap(2 * L + 2 * S)>();
    else if (ns == 1)
        wait_vm<vm_cap(2 * L + S)>();
    else
        wait_vm<2 * L>();
#else
    wait_vm<2 * L>();
#endif
}

// One 16-byte global-to-LDS transfer per lane: lane i's 16 bytes from src go
// to LDS byte address lds + 16 i.  Written out (the builtin makes the
// compiler wait for every transfer in flight before any LDS read, which
// would undo the prefetch); the kernel orders it itself with wait_vm and a
// barrier.  It has no register result.
__device__ __forceinline__ void dma16(const void *src, uint32_t lds) {
    asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off" : : "v"(src), "s"(lds) : "memory", "m0");
}

// This lane's source element offsets for the transfers of one staged row at
// row 0 of the item's tile (the row yi adds yi nx CI), -1 where the position
// is padding or its voxel lies outside the volume in x or z.
template <int CI, int NW = 4, int XW = 34> struct ConvDmaOff {
    long off[ConvLds<CI, NW, XW>::L];
};
template <int CI, int NW = 4, int XW = 34>
__device__ __forceinline__ void conv_dma_prep(ConvDmaOff<CI, NW, XW> &O, const Dims &d, int x0, int z0, int w,
                                              int lane) {
    using G = ConvLds<CI, NW, XW>;
#pragma unroll
    for (int i = 0; i < G::L; ++i) {
        const int k = i * NW + w, p = k * 64 + lane;
        const int zi = p / (XW * G::CP), xi = (p / G::CP) % XW, qs = p % G::CP;
        const int q = conv_perm<CI, NW>(xi, qs);  // the chunk that slot holds
        const int zz = z0 - 1 + zi, xx = x0 - 1 + xi;
        const bool ok = p < G::P && q < G::C && zz >= 0 && zz < d.nz && xx >= 0 && xx < d.nx;
        O.off[i] = ok ? ((long)zz * d.ny * d.nx + xx) * CI + q * 8 : -1;
    }
}

template <int CI, int NW = 4, int XW = 34>
__device__ __forceinline__ void conv_dma_row(uint32_t slot, const uint16_t *__restrict__ X,
                                             const ConvDmaOff<CI, NW, XW> &O, const Dims &d, int yi, int w) {
    using G = ConvLds<CI, NW, XW>;
    const bool yok = yi >= 0 && yi < d.ny;  // wave-uniform
    const long yoff = (long)yi * d.nx * CI;
#pragma unroll
    for (int i = 0; i < G::L; ++i) {
        const uint16_t *src = yok && O.off[i] >= 0 ? X + (O.off[i] + yoff) : kConvZeros;
        dma16(src, slot + (uint32_t)((i * NW + w) * 1024));
    }
}

// The MFMAs of one staged row for the wave's z (slot row w + dz) with the
// epilogue of the row completed one step earlier (accumulator aF, output
// row yo) interleaved between them: its GELU, BF16 conversion and stores
// issue while the matrix pipe works on this row.  The accumulator of row
// YI + 1 (the one stored a step earlier) is not cleared: its first MFMA
// takes the bias (the lane's output channel m) as the addend instead.
template <int CI, bool ZOUT, bool STORE>
__device__ __forceinline__ void conv_lds_mfma_epi(const uint16_t (&slot)[ConvLds<CI>::SLOT * 8], const ConvW<CI> &W,
                                                  int w, int m, int kh, floatx16 &aP, floatx16 &a0, floatx16 &aN,
                                                  floatx16 &aF, float bc, float *__restrict__ zout,
                                                  uint16_t *__restrict__ hout, const Dims &d, int x0, int yo,
                                                  int z) {
    using G = ConvLds<CI>;
    const long v0 = ((long)z * d.ny + yo) * d.nx + x0;
    // fragments of tap group g = (dz, dx), the next group's read while this one's MFMAs run
    auto frag = [&](int g, int kc) {
        const int dz = g / 3, dx = g % 3;
        return *reinterpret_cast<const bf16x8 *>(slot + (((w + dz) * 34) * G::CP + conv_slot<CI>(m + dx, kc * 2 + kh)) * 8);
    };
    // fragments two tap groups ahead of the MFMAs that use them
    bf16x8 fr[3][CI / 16];
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int kc = 0; kc < CI / 16; ++kc) fr[g][kc] = frag(g, kc);
#pragma unroll
    for (int g = 0; g < 9; ++g) {
        const int dz = g / 3, dx = g % 3;
        if (g < 7) {
#pragma unroll
            for (int kc = 0; kc < CI / 16; ++kc) fr[(g + 2) % 3][kc] = frag(g + 2, kc);
        }
#pragma unroll
        for (int kc = 0; kc < CI / 16; ++kc) {
            const bf16x8 a = fr[g % 3][kc];
            const int tb = dz * 9 + dx;
            // row YI + 1 starts here: its first product adds to the bias
            aN = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, W.f[tb][kc], g == 0 && kc == 0 ? (floatx16)bc : aN, 0,
                                                         0, 0);
            a0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, W.f[tb + 3][kc], a0, 0, 0, 0);
            aP = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, W.f[tb + 6][kc], aP, 0, 0, 0);
        }
        if (STORE) {
#pragma unroll
            for (int r = g * 16 / 9; r < (g + 1) * 16 / 9; ++r) {
                const long v = v0 + 8 * (r >> 2) + 4 * kh + (r & 3);
                const float zv = aF[r];
                if (ZOUT) zout[v * 32 + m] = zv;
                hout[v * 32 + m] = to_bf_cvt(gelu(zv));
            }
        }
    }
    // order: the first two groups' fragment reads; then per group the reads
    // for two groups ahead and its MFMAs, each followed by up to seven
    // vector instructions of the epilogue (they run in the shadow of the
    // matrix instruction before them)
    __builtin_amdgcn_sched_group_barrier(0x100, 2 * (CI / 16), 0);  // LDS reads
#pragma unroll
    for (int g = 0; g < 9; ++g) {
        if (g < 7) __builtin_amdgcn_sched_group_barrier(0x100, CI / 16, 0);
#pragma unroll
        for (int i = 0; i < 3 * (CI / 16); ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);             // MFMA
            if (STORE) __builtin_amdgcn_sched_group_barrier(0x002, 7, 0);  // VALU
        }
    }
}

template <bool ZOUT>
__device__ __forceinline__ void conv_lds_flush(const floatx16 &acc, float bc, float *__restrict__ zout,
                                               uint16_t *__restrict__ hout, const Dims &d, int x0, int yo, int z,
                                               int m, int kh) {
    const long v0 = ((long)z * d.ny + yo) * d.nx + x0;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const long v = v0 + 8 * (r >> 2) + 4 * kh + (r & 3);
        const float zv = acc[r];
        if (ZOUT) zout[v * 32 + m] = zv;
        hout[v * 32 + m] = to_bf_cvt(gelu(zv));
    }
}

// The 16-channel variant without the pre-activation output fits two blocks
// per CU (registers and LDS); the others hold more and run one.
template <int CI, bool ZOUT> constexpr int conv_lds_blocks() { return CI == 16 && !ZOUT ? MGCT_CONV16_BLOCKS : 1; }

template <int CI, bool ZOUT>
__global__ __launch_bounds__(256, (conv_lds_blocks<CI, ZOUT>())) void k_conv_lds(const uint16_t *__restrict__ X, const uint16_t *__restrict__ P,
                                                     const float *__restrict__ bias, float *__restrict__ zout,
                                                     uint16_t *__restrict__ hout, Dims d, int n_items) {
    using G = ConvLds<CI>;
    __shared__ __align__(16) uint16_t ring0[G::SLOT * 8], ring1[G::SLOT * 8], ring2[G::SLOT * 8],
        ring3[G::SLOT * 8];
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int m = lane & 31, kh = lane >> 5;
    // the slots' LDS byte addresses (a __shared__ address is its LDS offset in the low 32 bits)
    const uint32_t l0 = (uint32_t)(uintptr_t)ring0, l1 = (uint32_t)(uintptr_t)ring1,
                   l2 = (uint32_t)(uintptr_t)ring2, l3 = (uint32_t)(uintptr_t)ring3;
    ConvW<CI> W;
#pragma unroll
    for (int t = 0; t < 27; ++t)
#pragma unroll
        for (int kc = 0; kc < CI / 16; ++kc)
            W.f[t][kc] = *reinterpret_cast<const bf16x8 *>(P + ((long)t * 32 + m) * CI + kc * 16 + kh * 8);
    const float bc = bias[m];
    wait_vm<0>();  // weights and bias in registers before the first transfer
    const int nxt = d.nx / 32;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {  // block-uniform
        const int x0 = (it % nxt) * 32, z0 = (it / nxt) * 4, z = z0 + w;
        const bool live = z < d.nz;  // a wave past the grid still moves data and meets the barriers
        // accumulator of output row o: A[o mod 4]; ring slot of input row r: (r + 1) mod 4
        floatx16 A0{}, A1{}, A2{}, A3{};
        ConvDmaOff<CI> O;
        conv_dma_prep<CI>(O, d, x0, z0, w, lane);
        __syncthreads();  // the previous item's reads of the ring are done
        conv_dma_row<CI>(l0, X, O, d, -1, w);
        conv_dma_row<CI>(l1, X, O, d, 0, w);
        conv_dma_row<CI>(l2, X, O, d, 1, w);
        // step YI: its row from slot RS, the row three ahead into slot RN,
        // MFMAs into rows YI - 1 (AP), YI (A0_), YI + 1 (AN), the epilogue of
        // row YI - 2 (AF) interleaved
#define MGCT_CONV_STEP(RS, RN, YI, AP, A0_, AN, AF, STORE)                                                       \
    {                                                                                                            \
        conv_row_wait<G::L, (ZOUT ? 32 : 16)>((YI), live);                                                      \
        __syncthreads();                                                                                         \
        conv_dma_row<CI>(RN, X, O, d, (YI) + 3, w);                                                              \
        if (live)                                                                                                \
            conv_lds_mfma_epi<CI, ZOUT, STORE>(RS, W, w, m, kh, AP, A0_, AN, AF, bc, zout, hout, d, x0, (YI) - 2, \
                                                z);                                                              \
    }
        MGCT_CONV_STEP(ring0, l3, -1, A2, A3, A0, A1, false)
        if (0 <= d.ny) MGCT_CONV_STEP(ring1, l0, 0, A3, A0, A1, A2, false)
        if (1 <= d.ny) MGCT_CONV_STEP(ring2, l1, 1, A0, A1, A2, A3, false)
        if (2 <= d.ny) MGCT_CONV_STEP(ring3, l2, 2, A1, A2, A3, A0, true)
        for (int yi = 3; yi <= d.ny; yi += 4) {
            MGCT_CONV_STEP(ring0, l3, yi, A2, A3, A0, A1, true)
            if (yi + 1 > d.ny) break;
            MGCT_CONV_STEP(ring1, l0, yi + 1, A3, A0, A1, A2, true)
            if (yi + 2 > d.ny) break;
            MGCT_CONV_STEP(ring2, l1, yi + 2, A0, A1, A2, A3, true)
            if (yi + 3 > d.ny) break;
            MGCT_CONV_STEP(ring3, l2, yi + 3, A1, A2, A3, A0, true)
        }
#undef MGCT_CONV_STEP
        // the last row, ny - 1, completed in the last step
        if (live) {
            const int o = d.ny - 1;
            switch (o & 3) {
                case 0: conv_lds_flush<ZOUT>(A0, bc, zout, hout, d, x0, o, z, m, kh); break;
                case 1: conv_lds_flush<ZOUT>(A1, bc, zout, hout, d, x0, o, z, m, kh); break;
                case 2: conv_lds_flush<ZOUT>(A2, bc, zout, hout, d, x0, o, z, m, kh); break;
                default: conv_lds_flush<ZOUT>(A3, bc, zout, hout, d, x0, o, z, m, kh); break;
            }
        }
        wait_vm<0>();  // no transfer into the ring stays in flight past the item
    }
}

// Layer 3 (32 -> 32 channels) on large grids with eight waves per block.
// The same ring of staged input rows as k_conv_lds, but waves w and w + 4
// take the same z row (w mod 4), the first the output channels 0..15 and the
// second 16..31: each holds half the weights, so two waves fit on every SIMD
// and one issues while the other waits.  The products are 16x16x32 MFMAs,
// D[c][x] = sum over the 32 input channels of W[c][ci] X[ci][x] for the
// wave's 16 channels and 16 voxels of one half (hx) of the 32-voxel tile:
// lane (n, kg) = (lane mod 16, lane / 16) holds row n of a weight fragment
// (channel c0 + n, inputs 8 kg .. 8 kg + 7), column n of an input fragment
// (voxel hx 16 + n, the same inputs, chunk kg of the voxel in LDS), and of
// the result the channels c0 + 4 kg .. c0 + 4 kg + 3 of voxel hx 16 + n,
// which leave as one 8-byte store.  Accumulators of output row o: A[o mod 4],
// one 4-vector per half.
constexpr int kHwWaves = 8;
using ConvHwLds = ConvLds<32, kHwWaves>;

// The accumulator already holds the bias (the row's first MFMA starts from it).
template <bool ZOUT>
__device__ __forceinline__ void conv_hw_store(const floatx4 &zv, float *__restrict__ zout, uint16_t *__restrict__ hout,
                                              long e) {
    if (ZOUT) *reinterpret_cast<floatx4 *>(zout + e) = zv;
    *reinterpret_cast<uint2 *>(hout + e) =
        make_uint2(pack_bf16x2(gelu(zv[0]), gelu(zv[1])), pack_bf16x2(gelu(zv[2]), gelu(zv[3])));
}

// The MFMAs of one staged row for the wave's z (slot row wz + dz) into the
// rows YI - 1 (aP), YI (a0) and YI + 1 (aN, which starts here from the
// bias), with the epilogue of row yo = YI - 2 (aF) interleaved.
template <bool ZOUT, bool STORE>
__device__ __forceinline__ void conv_hw_mfma_epi(const uint16_t (&slot)[ConvHwLds::SLOT * 8], const bf16x8 (&W)[27],
                                                 int wz, int n, int kg, floatx4 (&aP)[2], floatx4 (&a0)[2],
                                                 floatx4 (&aN)[2], const floatx4 (&aF)[2], const floatx4 &bc,
                                                 float *__restrict__ zout, uint16_t *__restrict__ hout,
                                                 const Dims &d, int x0, int yo, int z, int c0) {
    auto frag = [&](int g, int hx) {
        const int dz = g / 3, dx = g % 3, xi = hx * 16 + n + dx;
        return *reinterpret_cast<const bf16x8 *>(slot + ((wz + dz) * 34 * 4 + conv_slot<32, kHwWaves>(xi, kg)) * 8);
    };
    const long e0 = (((long)z * d.ny + yo) * d.nx + x0 + n) * 32 + c0 + 4 * kg;
    // fragments two tap groups ahead of the MFMAs that use them
    bf16x8 fr[3][2];
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        fr[g][0] = frag(g, 0);
        fr[g][1] = frag(g, 1);
    }
#pragma unroll
    for (int g = 0; g < 9; ++g) {
        const int dz = g / 3, dx = g % 3, tb = dz * 9 + dx;
        if (g < 7) {
            fr[(g + 2) % 3][0] = frag(g + 2, 0);
            fr[(g + 2) % 3][1] = frag(g + 2, 1);
        }
#pragma unroll
        for (int hx = 0; hx < 2; ++hx) {
            const bf16x8 b = fr[g % 3][hx];
            aN[hx] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W[tb], b, g == 0 ? bc : aN[hx], 0, 0, 0);
            a0[hx] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W[tb + 3], b, a0[hx], 0, 0, 0);
            aP[hx] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W[tb + 6], b, aP[hx], 0, 0, 0);
        }
        if (STORE && (g == 2 || g == 6)) conv_hw_store<ZOUT>(aF[g / 4], zout, hout, e0 + (g / 4) * 16 * 32);
    }
    // order: the first two groups' fragment reads; then per group the reads
    // for two groups ahead and its six MFMAs, each followed by up to three
    // vector instructions of the epilogue
    __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);  // LDS reads
#pragma unroll
    for (int g = 0; g < 9; ++g) {
        if (g < 7) __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);             // MFMA
            if (STORE) __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);  // VALU
        }
    }
}

template <bool ZOUT>
__global__ __launch_bounds__(512, 1) void k_conv32_hw(const uint16_t *__restrict__ X, const uint16_t *__restrict__ P,
                                                      const float *__restrict__ bias, float *__restrict__ zout,
                                                      uint16_t *__restrict__ hout, Dims d, int n_items) {
    using G = ConvHwLds;
    __shared__ __align__(16) uint16_t ring0[G::SLOT * 8], ring1[G::SLOT * 8], ring2[G::SLOT * 8],
        ring3[G::SLOT * 8];
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wz = w & 3, c0 = (w >> 2) * 16, n = lane & 15, kg = lane >> 4;
    const uint32_t l0 = (uint32_t)(uintptr_t)ring0, l1 = (uint32_t)(uintptr_t)ring1,
                   l2 = (uint32_t)(uintptr_t)ring2, l3 = (uint32_t)(uintptr_t)ring3;
    bf16x8 W[27];
#pragma unroll
    for (int t = 0; t < 27; ++t) W[t] = *reinterpret_cast<const bf16x8 *>(P + ((long)t * 32 + c0 + n) * 32 + kg * 8);
    floatx4 bc;
#pragma unroll
    for (int r = 0; r < 4; ++r) bc[r] = bias[c0 + 4 * kg + r];
    wait_vm<0>();  // weights and bias in registers before the first transfer
    const int nxt = d.nx / 32;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {  // block-uniform
        const int x0 = (it % nxt) * 32, z0 = (it / nxt) * 4, z = z0 + wz;
        const bool live = z < d.nz;  // a wave past the grid still moves data and meets the barriers
        floatx4 A0[2] = {}, A1[2] = {}, A2[2] = {}, A3[2] = {};
        ConvDmaOff<32, kHwWaves> O;
        conv_dma_prep<32, kHwWaves>(O, d, x0, z0, w, lane);
        __syncthreads();  // the previous item's reads of the ring are done
        conv_dma_row<32, kHwWaves>(l0, X, O, d, -1, w);
        conv_dma_row<32, kHwWaves>(l1, X, O, d, 0, w);
        conv_dma_row<32, kHwWaves>(l2, X, O, d, 1, w);
#define MGCT_CONV_HW_STEP(RS, RN, YI, AP, A0_, AN, AF, STORE)                                                      \
    {                                                                                                            \
        conv_row_wait<G::L, (ZOUT ? 4 : 2)>((YI), live);                                                        \
        __syncthreads();                                                                                         \
        conv_dma_row<32, kHwWaves>(RN, X, O, d, (YI) + 3, w);                                                    \
        if (live)                                                                                                \
            conv_hw_mfma_epi<ZOUT, STORE>(RS, W, wz, n, kg, AP, A0_, AN, AF, bc, zout, hout, d, x0, (YI) - 2, z,  \
                                          c0);                                                                   \
    }
        MGCT_CONV_HW_STEP(ring0, l3, -1, A2, A3, A0, A1, false)
        if (0 <= d.ny) MGCT_CONV_HW_STEP(ring1, l0, 0, A3, A0, A1, A2, false)
        if (1 <= d.ny) MGCT_CONV_HW_STEP(ring2, l1, 1, A0, A1, A2, A3, false)
        if (2 <= d.ny) MGCT_CONV_HW_STEP(ring3, l2, 2, A1, A2, A3, A0, true)
        for (int yi = 3; yi <= d.ny; yi += 4) {
            MGCT_CONV_HW_STEP(ring0, l3, yi, A2, A3, A0, A1, true)
            if (yi + 1 > d.ny) break;
            MGCT_CONV_HW_STEP(ring1, l0, yi + 1, A3, A0, A1, A2, true)
            if (yi + 2 > d.ny) break;
            MGCT_CONV_HW_STEP(ring2, l1, yi + 2, A0, A1, A2, A3, true)
            if (yi + 3 > d.ny) break;
            MGCT_CONV_HW_STEP(ring3, l2, yi + 3, A1, A2, A3, A0, true)
        }
#undef MGCT_CONV_HW_STEP
        // the last row, ny - 1, completed in the last step
        if (live) {
            const int o = d.ny - 1;
            const long e0 = (((long)z * d.ny + o) * d.nx + x0 + n) * 32 + c0 + 4 * kg;
            const floatx4 *F = (o & 3) == 0 ? A0 : (o & 3) == 1 ? A1 : (o & 3) == 2 ? A2 : A3;
            conv_hw_store<ZOUT>(F[0], zout, hout, e0);
            conv_hw_store<ZOUT>(F[1], zout, hout, e0 + 16 * 32);
        }
        wait_vm<0>();  // no transfer into the ring stays in flight past the item
    }
}

// Layer 4 (32 channels -> 1) on the matrix cores.  For an input row the
// products of every input voxel with the weights of all nine in-plane taps
// (dx, dy) are one small GEMM: E[m][j] = sum over dz and channels of
// h3[x0 + m, yi, z + dz][c] W4[c][tap(j, dz)] (K = 3 x 32 in 16-channel
// chunks, N = 9 of 32 columns, each weight as a BF16 pair so that 16 bits of
// it are kept), whose result goes to LDS; output (x, yo) then adds
// E[x - x0 + dx][(dx, dy)] over dx for the row yo = yi - dy.  A wave's 32
// input voxels x0 .. x0 + 31 serve the 30 outputs x0 + 1 .. x0 + 30 (tiles at
// stride 30), marching up y with three output rows in flight.  A wave takes
// ZW consecutive output planes, whose ZW + 2 input slices per row it loads
// once; a block's 4 waves take 4 ZW consecutive z.  The kernel waits on
// memory latency, so it runs fastest with one plane per wave at 3 waves per
// SIMD: two planes per wave, a block of 8 one-plane waves, blocks ordered so
// that z neighbours share a die's L2 (all read fewer bytes) and register
// caps for more waves (they spill) each ran slower.  The next row's A fragments load while the
// current row is worked on.

// the input slices z0 - 1 .. z0 + ZW of one row for the wave's ZW output planes
template <int ZW> struct Conv4Row {
    bf16x8 a[ZW + 2][2];  // [slice][channel chunk]
};

template <int ZW>
__device__ __forceinline__ void conv4_load(Conv4Row<ZW> &R, const uint16_t *__restrict__ h3, const Dims &d, int x,
                                           int z0, int yi, int kh) {
#pragma unroll
    for (int sl = 0; sl < ZW + 2; ++sl) {
        const int zz = z0 + sl - 1;
        const bool ok = yi >= 0 && yi < d.ny && zz >= 0 && zz < d.nz && x >= 0 && x < d.nx;
        const uint16_t *src = (ok ? h3 + (((long)zz * d.ny + yi) * d.nx + x) * 32 : kConvZeros) + kh * 8;
#pragma unroll
        for (int kc = 0; kc < 2; ++kc) R.a[sl][kc] = *reinterpret_cast<const bf16x8 *>(src + (ok ? kc * 16 : 0));
    }
}

#ifndef MGCT_CONV4_ZW
#define MGCT_CONV4_ZW 1
#endif
constexpr int kConv4Zw = MGCT_CONV4_ZW;  // output planes per wave; a block's 4 waves take 4 kConv4Zw planes

template <int ZW>
__global__ __launch_bounds__(256) void k_conv4_ym(const uint16_t *__restrict__ h3, const uint16_t *__restrict__ P4,
                                                  const float *__restrict__ w, const float *__restrict__ u,
                                                  float *__restrict__ out, Dims d) {
    __shared__ float E[4][ZW][32 * 9];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = lane & 31, kh = lane >> 5;
    const int ntile = (d.nx + 29) / 30;
    const int x0 = (blockIdx.x % ntile) * 30 - 1, z0 = (blockIdx.x / ntile) * 4 * ZW + wv * ZW;
    if (z0 >= d.nz) return;  // whole wave; no barrier in this kernel
    bf16x8 Bf[2][3][2];
#pragma unroll
    for (int hl = 0; hl < 2; ++hl)
#pragma unroll
        for (int dz = 0; dz < 3; ++dz)
#pragma unroll
            for (int kc = 0; kc < 2; ++kc)
                Bf[hl][dz][kc] =
                    *reinterpret_cast<const bf16x8 *>(P4 + ((((hl * 3 + dz) * 2 + kc) * 32 + m) * 16 + kh * 8));
    const float b4 = w[kB4];
    const int xo = x0 + 1 + m;                   // this lane's output x (lanes m < 30, kh = 0)
    const bool gather = kh == 0 && m < 30 && xo < d.nx;
    float oP[ZW], o0[ZW], oN[ZW];                // per plane: output rows yi - 1, yi, yi + 1
#pragma unroll
    for (int q = 0; q < ZW; ++q) oP[q] = o0[q] = oN[q] = 0.f;
    // one input row from buffer C (the next row's loads already in flight)
    auto row = [&](const Conv4Row<ZW> &C, int yi) {
#pragma unroll
        for (int q = 0; q < ZW; ++q) {
            floatx16 acc{};
#pragma unroll
            for (int dz = 0; dz < 3; ++dz)
#pragma unroll
                for (int kc = 0; kc < 2; ++kc)
#pragma unroll
                    for (int hl = 0; hl < 2; ++hl)
                        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(C.a[q + dz][kc], Bf[hl][dz][kc], acc, 0, 0, 0);
            if (m < 9) {
#pragma unroll
                for (int r = 0; r < 16; ++r) E[wv][q][(8 * (r >> 2) + 4 * kh + (r & 3)) * 9 + m] = acc[r];
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (gather) {
#pragma unroll
            for (int q = 0; q < ZW; ++q) {
                // slot j = 3 (dy + 1) + dx + 1 of input m + 1 + dx
                const float *e = &E[wv][q][(m + 1) * 9];
                oN[q] += e[-9 + 0] + e[1] + e[9 + 2];   // dy = -1 -> output row yi + 1
                o0[q] += e[-9 + 3] + e[4] + e[9 + 5];   // dy = 0
                oP[q] += e[-9 + 6] + e[7] + e[9 + 8];   // dy = +1 -> output row yi - 1
            }
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int q = 0; q < ZW; ++q) {
            if (gather && yi - 1 >= 0 && z0 + q < d.nz) {
                const long v = ((long)(z0 + q) * d.ny + (yi - 1)) * d.nx + xo;
                out[v] = u[v] + (oP[q] + b4);
            }
            oP[q] = o0[q];
            o0[q] = oN[q];
            oN[q] = 0.f;
        }
    };
    Conv4Row<ZW> RA, RB;
    conv4_load<ZW>(RA, h3, d, x0 + m, z0, -1, kh);
    for (int yi = -1; yi <= d.ny; yi += 2) {
        conv4_load<ZW>(RB, h3, d, x0 + m, z0, yi + 1, kh);
        row(RA, yi);
        if (yi + 1 > d.ny) break;
        conv4_load<ZW>(RA, h3, d, x0 + m, z0, yi + 2, kh);
        row(RB, yi + 1);
    }
}

// Layer 4 on large grids with its input rows staged like layers 2 and 3
// (k_conv_lds: a 4-slot LDS ring filled by global-to-LDS transfers three
// rows ahead, one barrier per row): a block takes 30 output x (x0 .. x0 + 29,
// tiles at stride 30; the ring holds the 32 voxels x0 - 1 .. x0 + 30 of the
// 6 z rows z0 - 1 .. z0 + 4) and 4 consecutive z, one wave per z.  Per input
// row a wave forms the tap products E of k_conv4_ym from the ring's fragments,
// gathers them for its 30 outputs and stores the output row this input row
// completes.  The wait before a row leaves the two later rows' transfers
// outstanding (it also waits for the few output loads and stores issued
// between them, which vector memory completes in order).
using Conv4Lds = ConvLds<32, 4, 32>;

__device__ __forceinline__ void conv4_lds_row(const uint16_t (&slot)[Conv4Lds::SLOT * 8], const bf16x8 (&Bf)[2][3][2],
                                              int wv, int m, int kh, bool gather, float *Ew, float &oP, float &o0,
                                              float &oN) {
    floatx16 acc{};
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
        for (int kc = 0; kc < 2; ++kc) {
            const bf16x8 a =
                *reinterpret_cast<const bf16x8 *>(slot + ((wv + dz) * Conv4Lds::X * 4 + conv_slot<32>(m, kc * 2 + kh)) * 8);
#pragma unroll
            for (int hl = 0; hl < 2; ++hl) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, Bf[hl][dz][kc], acc, 0, 0, 0);
        }
    if (m < 9) {
#pragma unroll
        for (int r = 0; r < 16; ++r) Ew[(8 * (r >> 2) + 4 * kh + (r & 3)) * 9 + m] = acc[r];
    }
    __builtin_amdgcn_wave_barrier();
    if (gather) {
        // slot j = 3 (dy + 1) + dx + 1 of staged input m + 1 + dx
        const float *e = Ew + (m + 1) * 9;
        oN += e[-9 + 0] + e[1] + e[9 + 2];  // dy = -1 -> output row yi + 1
        o0 += e[-9 + 3] + e[4] + e[9 + 5];  // dy = 0
        oP += e[-9 + 6] + e[7] + e[9 + 8];  // dy = +1 -> output row yi - 1
    }
    __builtin_amdgcn_wave_barrier();
}

__global__ __launch_bounds__(256) void k_conv4_lds(const uint16_t *__restrict__ h3, const uint16_t *__restrict__ P4,
                                                   const float *__restrict__ w, const float *__restrict__ u,
                                                   float *__restrict__ out, Dims d, int n_items) {
    using G = Conv4Lds;
    __shared__ __align__(16) uint16_t ring0[G::SLOT * 8], ring1[G::SLOT * 8], ring2[G::SLOT * 8],
        ring3[G::SLOT * 8];
    __shared__ float E[4][32 * 9];
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int m = lane & 31, kh = lane >> 5;
    const uint32_t l0 = (uint32_t)(uintptr_t)ring0, l1 = (uint32_t)(uintptr_t)ring1,
                   l2 = (uint32_t)(uintptr_t)ring2, l3 = (uint32_t)(uintptr_t)ring3;
    bf16x8 Bf[2][3][2];
#pragma unroll
    for (int hl = 0; hl < 2; ++hl)
#pragma unroll
        for (int dz = 0; dz < 3; ++dz)
#pragma unroll
            for (int kc = 0; kc < 2; ++kc)
                Bf[hl][dz][kc] =
                    *reinterpret_cast<const bf16x8 *>(P4 + ((((hl * 3 + dz) * 2 + kc) * 32 + m) * 16 + kh * 8));
    const float b4 = w[kB4];
    wait_vm<0>();  // weights in registers before the first transfer
    float *Ew = E[wv];
    const int ntile = (d.nx + 29) / 30;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {  // block-uniform
        const int x0 = (it % ntile) * 30, z0 = (it / ntile) * 4, z = z0 + wv;
        const bool live = z < d.nz;  // a wave past the grid still moves data and meets the barriers
        const int xo = x0 + m;       // this lane's output x (lanes m < 30, kh = 0)
        const bool gather = kh == 0 && m < 30 && xo < d.nx;
        float oP = 0.f, o0 = 0.f, oN = 0.f;  // output rows yi - 1, yi, yi + 1
        ConvDmaOff<32, 4, 32> O;
        conv_dma_prep<32, 4, 32>(O, d, x0, z0, wv, lane);
        __syncthreads();  // the previous item's reads of the ring are done
        conv_dma_row<32, 4, 32>(l0, h3, O, d, -1, wv);
        conv_dma_row<32, 4, 32>(l1, h3, O, d, 0, wv);
        conv_dma_row<32, 4, 32>(l2, h3, O, d, 1, wv);
        // step YI: input row YI from slot RS, row YI + 3 into slot RN; stores
        // the completed output row YI - 1
#define MGCT_CONV4_STEP(RS, RN, YI)                                                                              \
    {                                                                                                            \
        wait_vm<2 * G::L>();                                                                                     \
        __syncthreads();                                                                                         \
        conv_dma_row<32, 4, 32>(RN, h3, O, d, (YI) + 3, wv);                                                     \
        if (live) {                                                                                              \
            conv4_lds_row(RS, Bf, wv, m, kh, gather, Ew, oP, o0, oN);                                            \
            if (gather && (YI) >= 1) {                                                                           \
                const long v = ((long)z * d.ny + ((YI) - 1)) * d.nx + xo;                                        \
                out[v] = u[v] + (oP + b4);                                                                       \
            }                                                                                                    \
            oP = o0;                                                                                             \
            o0 = oN;                                                                                             \
            oN = 0.f;                                                                                            \
        }                                                                                                        \
    }
        MGCT_CONV4_STEP(ring0, l3, -1)
        for (int yi = 0; yi <= d.ny; yi += 4) {
            MGCT_CONV4_STEP(ring1, l0, yi)
            if (yi + 1 > d.ny) break;
            MGCT_CONV4_STEP(ring2, l1, yi + 1)
            if (yi + 2 > d.ny) break;
            MGCT_CONV4_STEP(ring3, l2, yi + 2)
            if (yi + 3 > d.ny) break;
            MGCT_CONV4_STEP(ring0, l3, yi + 3)
        }
#undef MGCT_CONV4_STEP
        wait_vm<0>();  // no transfer into the ring stays in flight past the item
    }
}

#ifndef MGCT_CONV_LDS
#define MGCT_CONV_LDS 1
#endif
// launch of either convolution kernel
#ifndef MGCT_CONV_DMA
#define MGCT_CONV_DMA 1  // large-grid forward: input rows staged in LDS by global-to-LDS loads
#endif
#ifndef MGCT_CONV4_LDS
#define MGCT_CONV4_LDS 1  // layer 4 on large grids from the LDS ring
#endif
#ifndef MGCT_CONV4_LDS_BLOCKS
#define MGCT_CONV4_LDS_BLOCKS 3  // persistent blocks per CU
#endif
#ifndef MGCT_CONV32_HW
#define MGCT_CONV32_HW 1  // the 32-channel layer on large grids: eight waves, half the channels each
#endif
#ifndef MGCT_CONV_YM_MIN_VOX
#define MGCT_CONV_YM_MIN_VOX (128L * 128 * 128)  // forward on the marching kernel from this many voxels
#endif
template <int CI, int MODE>
static void launch_conv(const uint16_t *X, const uint16_t *P, const float *bias, const float *zprev, float *zout,
                        uint16_t *hout, int nout, Dims d, hipStream_t s) {
    if (MODE == 0 && (long)d.nx * d.ny * d.nz >= MGCT_CONV_YM_MIN_VOX) {
        static int n_cu = 0;
        if (!n_cu) {
            int dev = 0;
            hipDeviceProp_t prop;
            n_cu = (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
                       ? prop.multiProcessorCount
                       : 256;
        }
        const int n_items = (d.nx / 32) * ((d.nz + 3) / 4);
        if (CI == 32 && MGCT_CONV32_HW) {
            const unsigned nb = (unsigned)std::min(n_items, n_cu);
            if (zout)
                k_conv32_hw<true><<<nb, 512, 0, s>>>(X, P, bias, zout, hout, d, n_items);
            else
                k_conv32_hw<false><<<nb, 512, 0, s>>>(X, P, bias, zout, hout, d, n_items);
        } else if (MGCT_CONV_DMA && zout)
            k_conv_lds<CI, true><<<(unsigned)std::min(n_items, n_cu * conv_lds_blocks<CI, true>()), 256, 0, s>>>(
                X, P, bias, zout, hout, d, n_items);
        else if (MGCT_CONV_DMA)
            k_conv_lds<CI, false><<<(unsigned)std::min(n_items, n_cu * conv_lds_blocks<CI, false>()), 256, 0, s>>>(
                X, P, bias, zout, hout, d, n_items);
        else
            k_conv_ym<CI><<<(unsigned)std::min(n_items, n_cu), 256, 0, s>>>(X, P, bias, zout, hout, d, n_items);
        return;
    }
    if (MGCT_CONV_LDS) {
        constexpr int YB = 4 * kConvLdsRows;
        const unsigned nb = (unsigned)((long)(d.nx / 32) * ((d.ny + YB - 1) / YB) * d.nz);
        const size_t lds = (size_t)3 * (YB + 2) * 34 * (CI + 8) * sizeof(uint16_t);
        k_conv_mfma_lds<CI, MODE><<<nb, 256, lds, s>>>(X, P, bias, zprev, zout, hout, nout, d);
    } else {
        const long w = (long)(d.nx / 32) * ((d.ny + kConvRows - 1) / kConvRows) * d.nz;
        k_conv_mfma<CI, MODE><<<(unsigned)((w + 3) / 4), 256, 0, s>>>(X, P, bias, zprev, zout, hout, nout, d);
    }
}

// channels-last BF16 [v][C] -> channels-first [C][nz+2][ny+2][nx+2] (zero border)
__global__ void k_to_cf_padded(const uint16_t *__restrict__ x, uint16_t *__restrict__ xt, int C, Dims d) {
    const long n = (long)d.nx * d.ny * d.nz;
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= n * C) return;
    const long v = i / C;
    const int c = (int)(i % C);
    int xx, yy, zz;
    split3(v, d.nx, d.ny, xx, yy, zz);
    const long PX = d.nx + 2, PY = d.ny + 2, PZ = d.nz + 2;
    xt[(((long)c * PZ + zz + 1) * PY + yy + 1) * PX + xx + 1] = x[i];
}

// channels-last BF16 [v][C] -> channels-first [C][v]
__global__ void k_to_cf(const uint16_t *__restrict__ x, uint16_t *__restrict__ xt, int C, long n) {
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= n * C) return;
    const long v = i / C;
    const int c = (int)(i % C);
    xt[(long)c * n + v] = x[i];
}

// dW[t][co][ci] partial over a chunk of rows: sum_v G[co][v] X[ci][v + off_t]
// (G channels-first [32][n], X channels-first padded [CI][nz+2][ny+2][nx+2]).
// One wave per (dy, dz, chunk) computes the three taps dx = -1, 0, 1: each
// G fragment is loaded once and used for the three shifted X fragments.
// K = 16 voxels per MFMA along x (nx % 16 == 0).
// partial[chunk][t][co][ci] (32 x 32, ci >= CI left zero).
template <int CI>
__global__ __launch_bounds__(256) void k_wgrad_mfma(const uint16_t *__restrict__ G, const uint16_t *__restrict__ X,
                                                    float *__restrict__ partial, Dims d, int rows_per_chunk,
                                                    int nchunks) {
    const int lane = threadIdx.x & 63;
    const long wid = blockIdx.x * 4L + (threadIdx.x >> 6);
    if (wid >= 9L * nchunks) return;  // whole wave; no barrier below
    const int tg = (int)(wid % 9), chunk = (int)(wid / 9);  // tg = 3 (dz + 1) + (dy + 1)
    const int m = lane & 31, kh = lane >> 5;
    const int dy = tg % 3 - 1, dz = tg / 3 - 1;
    const long n = (long)d.nx * d.ny * d.nz;
    const long PX = d.nx + 2, PY = d.ny + 2, PZ = d.nz + 2;
    const int nrows = d.ny * d.nz;
    const int r0 = chunk * rows_per_chunk, r1 = min(nrows, r0 + rows_per_chunk);
    floatx16 acc[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) acc[k] = floatx16{};
    for (int row = r0; row < r1; ++row) {
        const int y = row % d.ny, z = row / d.ny;
        const long vrow = (long)row * d.nx;
        // X row (ci = m) at x = -1 (padded index 0)
        const long prow = (((long)m * PZ + z + 1 + dz) * PY + y + 1 + dy) * PX;
        for (int x0 = 0; x0 < d.nx; x0 += 16) {
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(G + (long)m * n + vrow + x0 + kh * 8);
#pragma unroll
            for (int k = 0; k < 3; ++k) {  // dx = k - 1
                bf16x8 b = {};
                if (m < CI) {
                    const uint16_t *src = X + prow + k + x0 + kh * 8;
                    __builtin_memcpy(&b, __builtin_assume_aligned(src, 2), 16);
                }
                acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[k], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int t = 9 * (dz + 1) + 3 * (dy + 1) + k;  // tap index: t % 3 = dx + 1
        float *dst = partial + ((long)chunk * 27 + t) * 1024;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = 8 * (r >> 2) + 4 * kh + (r & 3);  // co
            dst[row * 32 + m] = acc[k][r];                     // ci = m
        }
    }
}

// grads[W at layer offset][co][ci][t] = sum_chunks partial[chunk][t][co][ci],
// one wave per weight as in k_sum_partials.
__global__ __launch_bounds__(256) void k_wgrad_mfma_sum(const float *__restrict__ partial, int nchunks, int CI,
                                                        float *__restrict__ gw) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);  // over co*CI*27
    if (i >= 32 * CI * 27) return;                      // whole wave
    const int co = i / (CI * 27), ci = (i / 27) % CI, t = i % 27;
    double acc = 0.0;
    for (int c = lane; c < nchunks; c += 64) acc += (double)partial[((long)c * 27 + t) * 1024 + co * 32 + ci];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) gw[i] = (float)acc;
}

__global__ __launch_bounds__(256) void k_bias_grad(const uint16_t *__restrict__ g, int C, long n, long chunk,
                                                   float *__restrict__ partial) {
    // thread (voxel group vg, channel c), C divides 256: coalesced rows of g
    const int c = threadIdx.x % C, vg = threadIdx.x / C, ng = 256 / C;
    const long v0 = blockIdx.x * chunk, v1 = min(n, v0 + chunk);
    double acc = 0.0;
    for (long v = v0 + vg; v < v1; v += ng) acc += (double)bf(g[v * C + c]);
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    if (vg == 0) {
        for (int k = 1; k < ng; ++k) acc += red[k * C + c];
        partial[blockIdx.x * (long)C + c] = (float)acc;
    }
}

__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       int n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ------------------------------------------------------------ drivers ----

static unsigned blocks(long n, int per = 256) { return (unsigned)((n + per - 1) / per); }

hipError_t cnn_pack(CnnState &S, hipStream_t s) {
    k_pack_weights<<<blocks(27 * 32 * 32), 256, 0, s>>>(S.master, S.p2f, S.p3f, S.p3d, S.p2d);
    k_pack_weights4<<<blocks(2 * 3 * 2 * 32 * 16), 256, 0, s>>>(S.master, S.p4);
    k_pack_weights1<<<blocks(3 * 16 * 32), 256, 0, s>>>(S.master, S.p1);
    return hipGetLastError();
}

hipError_t cnn_forward(CnnState &S, const CnnBuffers &B, const float *u, float *out, int nx, int ny, int nz,
                       bool keep, hipStream_t s) {
    const Dims d{nx, ny, nz};
    const long n = (long)nx * ny * nz;
    const unsigned vb = blocks(n);
    k_pad_input<<<(unsigned)((long)(ny + 2) * (nz + 2)), 256, 0, s>>>(u, B.up, d);
    k_conv1_mfma<<<blocks((long)ny * nz, 4), 256, 0, s>>>(B.up, S.p1, S.master, keep ? B.z1 : nullptr, B.h1, d);
    launch_conv<16, 0>(B.h1, S.p2f, S.master + kB2, nullptr, keep ? B.z2 : nullptr, B.h2, 32, d, s);
    launch_conv<32, 0>(B.h2, S.p3f, S.master + kB3, nullptr, keep ? B.z3 : nullptr, B.h3, 32, d, s);
    if (n >= MGCT_CONV_YM_MIN_VOX && MGCT_CONV4_LDS) {
        static int n_cu4 = 0;
        if (!n_cu4) {
            int dev = 0;
            hipDeviceProp_t prop;
            n_cu4 = (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
                        ? prop.multiProcessorCount
                        : 256;
        }
        const int n_items = ((nx + 29) / 30) * ((nz + 3) / 4);
        k_conv4_lds<<<(unsigned)std::min(n_items, MGCT_CONV4_LDS_BLOCKS * n_cu4), 256, 0, s>>>(B.h3, S.p4, S.master,
                                                                                               u, out, d, n_items);
    } else if (n >= MGCT_CONV_YM_MIN_VOX)
        k_conv4_ym<kConv4Zw><<<(unsigned)(((nx + 29) / 30) * ((nz + 4 * kConv4Zw - 1) / (4 * kConv4Zw))), 256, 0, s>>>(
            B.h3, S.p4, S.master, u, out, d);
    else
        k_conv4_fwd<<<vb, 256, 0, s>>>(B.h3, S.master, u, out, d);
    return hipGetLastError();
}

hipError_t cnn_backward(CnnState &S, const CnnBuffers &B, const float *u, const float *out, const float *target,
                        float *grads, double *loss_partials, int n_loss_blocks, int nx, int ny, int nz,
                        hipStream_t s) {
    const Dims d{nx, ny, nz};
    const long n = (long)nx * ny * nz;
    const unsigned vb = blocks(n);
    // dout = d loss / d out: from the mean squared error against target, or
    // (target NULL) already in B.dout
    if (target) k_mse<<<n_loss_blocks, 256, 0, s>>>(out, target, B.dout, loss_partials, n);
    // layer 4
    // bias gradients: blocks of 512 voxels (at most 4096 blocks), then a wave per channel
    const long vchunk = std::max(512L, (n + 4095) / 4096);
    const int nvb = (int)((n + vchunk - 1) / vchunk);
    const int rows = ny * nz;
    const int wrpc = 4, nwb = (nx / 32) * ((rows + wrpc - 1) / wrpc);
    k_wgrad_valu<4><<<nwb, 256, 0, s>>>(nullptr, B.h3, nullptr, B.dout, B.partial, d, wrpc);
    k_sum_partials<<<blocks(865, 4), 256, 0, s>>>(B.partial, nwb, 865, grads + kW4);
    k_conv4_bwd_input<<<vb, 256, 0, s>>>(B.dout, S.master, B.z3, B.dz3, d);
    // layer 3: weights (channels-first copies), bias, input gradient -> dz2
    const int rpc = 16, nch = (rows + rpc - 1) / rpc;
    k_to_cf<<<blocks(n * 32), 256, 0, s>>>(B.dz3, B.gT, 32, n);
    k_to_cf_padded<<<blocks(n * 32), 256, 0, s>>>(B.h2, B.xT, 32, d);
    k_wgrad_mfma<32><<<(unsigned)((9L * nch + 3) / 4), 256, 0, s>>>(B.gT, B.xT, B.partial, d, rpc, nch);
    k_wgrad_mfma_sum<<<blocks(32 * 32 * 27, 4), 256, 0, s>>>(B.partial, nch, 32, grads + kW3);
    k_bias_grad<<<nvb, 256, 0, s>>>(B.dz3, 32, n, vchunk, B.partial);
    k_sum_partials<<<blocks(32, 4), 256, 0, s>>>(B.partial, nvb, 32, grads + kB3);
    launch_conv<32, 1>(B.dz3, S.p3d, nullptr, B.z2, nullptr, B.dz2, 32, d, s);
    // layer 2
    k_to_cf<<<blocks(n * 32), 256, 0, s>>>(B.dz2, B.gT, 32, n);
    k_to_cf_padded<<<blocks(n * 16), 256, 0, s>>>(B.h1, B.xT, 16, d);
    k_wgrad_mfma<16><<<(unsigned)((9L * nch + 3) / 4), 256, 0, s>>>(B.gT, B.xT, B.partial, d, rpc, nch);
    k_wgrad_mfma_sum<<<blocks(32 * 16 * 27, 4), 256, 0, s>>>(B.partial, nch, 16, grads + kW2);
    k_bias_grad<<<nvb, 256, 0, s>>>(B.dz2, 32, n, vchunk, B.partial);
    k_sum_partials<<<blocks(32, 4), 256, 0, s>>>(B.partial, nvb, 32, grads + kB2);
    launch_conv<32, 1>(B.dz2, S.p2d, nullptr, B.z1, nullptr, B.dz1, 16, d, s);
    // layer 1 (input gradient not needed); dz1 holds GELU' * dh1 in BF16
    k_wgrad_valu<1><<<nwb, 256, 0, s>>>(u, nullptr, B.dz1, nullptr, B.partial, d, wrpc);
    k_sum_partials<<<blocks(448, 4), 256, 0, s>>>(B.partial, nwb, 448, grads + kW1);
    return hipGetLastError();
}

hipError_t cnn_adam(CnnState &S, const float *grads, float lr, hipStream_t s) {
    S.adam_t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)S.adam_t), c2 = 1.f - powf(b2, (float)S.adam_t);
    k_adam<<<blocks(kCnnParams), 256, 0, s>>>(S.master, grads, S.adam_m, S.adam_v, kCnnParams, lr, b1, b2, 1e-8f, c1,
                                              c2);
    return cnn_pack(S, s);
}

}  // namespace mgct
