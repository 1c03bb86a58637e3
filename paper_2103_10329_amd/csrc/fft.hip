// Fourier-space preconditioner: out = IDFT3(DFT3(in) * H(rho)), with the
// 3-D DFT sized to the grid (circular convolution), for power-of-two edges.
//
// Five passes over the volume, each batching whole lines of one axis in LDS
// (radix-2/4 Stockham, ping-pong buffers, up to 1024 complex values per block,
// fewer when that keeps at least 2048 blocks in flight):
//   1. along x: real input -> complex work array (forward)
//   2. along y: forward
//   3. along z: forward, multiply by H, inverse (same lines, one kernel)
//   4. along y: inverse
//   5. along x: inverse -> real output, scaled by 1/(nx ny nz)
// Lines along y and z are strided in memory; a block takes consecutive x so
// that global loads and stores stay coalesced.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <vector>

#include "mgct_internal.h"

namespace mgct {

// complex values per block, on the strided axes and on the contiguous x axis (512^3 filter: 8.66 ms with
// 4096 / 4096, 7.16 with 2048 / 2048, 6.66 with 2048 / 1024; with the die-grouped order of the strided passes
// 5.67 with 2048 / 1024, 5.46 with 1024 / 1024, 7.17 with 512 / 1024, 7.05 with 4096 / 1024)
constexpr int kFftElems = 1024;
constexpr int kFftElemsContig = 1024;

bool fft_size_ok(int n) { return n >= 2 && n <= 1024 && (n & (n - 1)) == 0; }

void host_twiddles(int n, std::vector<float2> &tw) {
    tw.resize(n / 2 > 0 ? n / 2 : 1);
    for (int k = 0; k < n / 2; ++k) {
        double ang = -2.0 * M_PI * (double)k / (double)n;
        tw[k] = make_float2((float)cos(ang), (float)sin(ang));
    }
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// In-LDS Stockham FFT of B lines of length N = 2^logN.  A stage of radix R
// takes the sub-transforms of length Ns to length R Ns: element j of a line
// (j < N/R, k = j mod Ns) combines src[j + r N/R] (r < R) after the twiddles
// exp(-+2 pi i r k/(R Ns)) by a length-R DFT and writes them to
// dst[(j - k) R + k + r Ns].  Lines of 128 points or more use radix-4 stages
// after one radix-2 stage when logN is odd (half the barriers and LDS round
// trips; 128^3 filter 0.123 -> 0.112 ms), shorter ones radix 2 throughout
// (radix 4 was slower at 64 points).  dir = +1 forward (exp(-2 pi i ...)),
// -1 inverse (unscaled).  tw[m] = exp(-2 pi i m/N) for m < N/2 (the other half
// is its negative).  Returns the buffer holding the result.
__device__ __forceinline__ float2 twiddle(const float2 *__restrict__ tw, int m, int half, int dir) {
    float2 w = m < half ? tw[m] : make_float2(-tw[m - half].x, -tw[m - half].y);
    if (dir < 0) w.y = -w.y;
    return w;
}

__device__ float2 *fft_lines(float2 *src, float2 *dst, int logN, int B, const float2 *__restrict__ tw, int dir) {
    const int N = 1 << logN, half = N >> 1;
    const bool r4 = logN >= 7;
    int lns = 0;  // log2 of the current sub-transform length Ns
    const int n2 = r4 ? (logN & 1) : logN;  // radix-2 stages
    for (; lns < n2; ++lns) {
        const int Ns = 1 << lns;
        for (int q = threadIdx.x; q < B * half; q += blockDim.x) {
            const int l = q >> (logN - 1);
            const int j = q & (half - 1);
            const int k = j & (Ns - 1);
            const float2 a = src[l * N + j];
            float2 w = tw[k << (logN - 1 - lns)];  // index below N/2
            if (dir < 0) w.y = -w.y;
            const float2 b = cmul(src[l * N + j + half], w);
            const int idx = ((j - k) << 1) + k;
            dst[l * N + idx] = make_float2(a.x + b.x, a.y + b.y);
            dst[l * N + idx + Ns] = make_float2(a.x - b.x, a.y - b.y);
        }
        __syncthreads();
        float2 *t = src;
        src = dst;
        dst = t;
    }
    const int quarter = N >> 2;
    for (; lns < logN; lns += 2) {
        const int Ns = 1 << lns;
        for (int q = threadIdx.x; q < B * quarter; q += blockDim.x) {
            const int l = q >> (logN - 2);
            const int j = q & (quarter - 1);
            const int k = j & (Ns - 1);
            const int step = k << (logN - 2 - lns);  // twiddle index of r = 1
            const float2 *in = src + l * N + j;
            const float2 v0 = in[0];
            const float2 v1 = cmul(in[quarter], twiddle(tw, step, half, dir));
            const float2 v2 = cmul(in[2 * quarter], twiddle(tw, 2 * step, half, dir));
            const float2 v3 = cmul(in[3 * quarter], twiddle(tw, 3 * step, half, dir));
            const float2 t0 = make_float2(v0.x + v2.x, v0.y + v2.y), t1 = make_float2(v0.x - v2.x, v0.y - v2.y);
            const float2 t2 = make_float2(v1.x + v3.x, v1.y + v3.y), d = make_float2(v1.x - v3.x, v1.y - v3.y);
            // (v1 - v3) times -i (forward) or +i (inverse)
            const float2 t3 = dir > 0 ? make_float2(d.y, -d.x) : make_float2(-d.y, d.x);
            float2 *out = dst + l * N + ((j - k) << 2) + k;
            out[0] = make_float2(t0.x + t2.x, t0.y + t2.y);
            out[Ns] = make_float2(t1.x + t3.x, t1.y + t3.y);
            out[2 * Ns] = make_float2(t0.x - t2.x, t0.y - t2.y);
            out[3 * Ns] = make_float2(t1.x - t3.x, t1.y - t3.y);
        }
        __syncthreads();
        float2 *t = src;
        src = dst;
        dst = t;
    }
    return src;
}

struct LineMap {
    long es;         // element stride
    int inner_log;   // lines are (outer, inner) with 2^inner_log inner lines per outer one;
    long inner_stride;  // base = outer*outer_stride + inner*inner_stride (shifts: every edge is a power of two)
    long outer_stride;
    __device__ long base(long L) const {
        return (L >> inner_log) * outer_stride + (L & ((1L << inner_log) - 1)) * inner_stride;
    }
};

struct RadialH {
    const float *table;
    int n_table;
    float rho_max;
    int nx, ny, nz;
    const float *hk;  // when set: the transfer function itself, [ez][ey][ex]
    int lognx, logny, lognz;
};

__device__ __forceinline__ float radial_gain(const RadialH &R, int ex, int ey, int ez) {
    if (R.hk) return R.hk[((long)ez * R.ny + ey) * R.nx + ex];
    const int kx = ex < (R.nx >> 1) ? ex : ex - R.nx;
    const int ky = ey < (R.ny >> 1) ? ey : ey - R.ny;
    const int kz = ez < (R.nz >> 1) ? ez : ez - R.nz;
    // k / n as an exact scaling by 2^-log n (n is a power of two)
    const float fx = ldexpf((float)kx, -R.lognx), fy = ldexpf((float)ky, -R.logny), fz = ldexpf((float)kz, -R.lognz);
    const float rho = 2.f * sqrtf(fx * fx + fy * fy + fz * fz);
    float t = rho / R.rho_max * (float)(R.n_table - 1);
    if (t >= (float)(R.n_table - 1)) return R.table[R.n_table - 1];
    const int i0 = (int)t;
    const float w = t - (float)i0;
    return fmaf(w, R.table[i0 + 1] - R.table[i0], R.table[i0]);
}

template <bool CONTIG, bool IN_REAL, bool OUT_REAL, bool MUL_H>
__global__ __launch_bounds__(256) void k_fft_pass(const float *__restrict__ in_r, const float2 *in_c,
                                                  float *__restrict__ out_r, float2 *out_c, int logN,
                                                  int logB, LineMap map, const float2 *__restrict__ tw, int dir,
                                                  float scale, RadialH R) {
    extern __shared__ float2 lds[];
    const int N = 1 << logN, B = 1 << logB, total = B * N;
    float2 *buf0 = lds, *buf1 = lds + total;
    // strided axes with at most 4 lines per block (runs of 32 bytes or less of
    // each 128-byte line): the blocks of one die take consecutive line groups
    // (the dispatcher hands blocks to the 8 dies in turn), so that the rest of
    // each line is read by a neighbour through the same L2 (512^3 filter
    // 6.66 -> 5.67 ms; with 8 lines per block, 128^3, it was 4 % slower)
    unsigned bi = blockIdx.x;
    if (!CONTIG && B <= 4 && (gridDim.x & 7u) == 0u) bi = (bi & 7u) * (gridDim.x >> 3) + (bi >> 3);
    const long L0 = (long)bi * B;
    for (int q = threadIdx.x; q < total; q += blockDim.x) {
        int l, e;
        if (CONTIG) { e = q & (N - 1); l = q >> logN; }
        else        { l = q & (B - 1); e = q >> logB; }
        const long g = map.base(L0 + l) + (long)e * map.es;
        buf0[l * N + e] = IN_REAL ? make_float2(in_r[g], 0.f) : in_c[g];
    }
    __syncthreads();
    float2 *res = fft_lines(buf0, buf1, logN, B, tw, dir);
    if (MUL_H) {
        // this pass runs along z: line L is (y, x) = (L / nx, L % nx)
        for (int q = threadIdx.x; q < total; q += blockDim.x) {
            const int l = q >> logN, e = q & (N - 1);
            const long L = L0 + l;
            const int ex = (int)(L & (R.nx - 1)), ey = (int)(L >> R.lognx);
            const float hgain = radial_gain(R, ex, ey, e);
            res[q] = make_float2(res[q].x * hgain, res[q].y * hgain);
        }
        __syncthreads();
        float2 *other = (res == buf0) ? buf1 : buf0;
        res = fft_lines(res, other, logN, B, tw, -dir);
    }
    for (int q = threadIdx.x; q < total; q += blockDim.x) {
        int l, e;
        if (CONTIG) { e = q & (N - 1); l = q >> logN; }
        else        { l = q & (B - 1); e = q >> logB; }
        const long g = map.base(L0 + l) + (long)e * map.es;
        const float2 v = res[l * N + e];
        if (OUT_REAL) out_r[g] = v.x * scale;
        else out_c[g] = v;
    }
}

static int ilog2(long n) {
    int l = 0;
    while ((1L << l) < n) ++l;
    return l;
}

hipError_t launch_radial_filter(const float *in, float *out, float2 *work, int nx, int ny, int nz, const float *table,
                                int n_table, float rho_max, const float2 *tw_all, hipStream_t s, const float *hk,
                                bool forward_only) {
    // tw_all holds the twiddles for nx, then ny, then nz (nx/2 + ny/2 + nz/2 entries)
    const float2 *twx = tw_all, *twy = tw_all + nx / 2, *twz = tw_all + nx / 2 + ny / 2;
    RadialH R{table, n_table, rho_max, nx, ny, nz, hk, ilog2(nx), ilog2(ny), ilog2(nz)};
    RadialH none{nullptr, 0, 1.f, nx, ny, nz, nullptr, ilog2(nx), ilog2(ny), ilog2(nz)};
    const long nvox = (long)nx * ny * nz;
    // lines per block: as many as fit kFftElems, fewer while that leaves
    // under 2048 blocks (down to 8 lines on strided axes, so that a block's
    // global accesses still cover 64 contiguous bytes)
    auto pick_B = [&](int n, long lines, bool strided) {
        long B = (strided ? kFftElems : kFftElemsContig) / n;
        if (B > lines) B = lines;
        const long bmin = strided ? 8 : 1;
        while (B > bmin && lines / B < 2048) B >>= 1;
        if (B < 1) B = 1;
        return ilog2(B);
    };
    auto lds_of = [](int logN, int logB) { return 2 * (sizeof(float2) << (logN + logB)); };
    auto threads_of = [](int logN, int logB) {
        const int half = 1 << (logN + logB - 1);
        return half >= 256 ? 256 : (half < 64 ? 64 : half);
    };
    // pass 1: x, real -> complex
    {
        const int logN = ilog2(nx), logB = pick_B(nx, (long)ny * nz, false);
        LineMap m{1, 40, nx, 0};
        const unsigned grid = (unsigned)(((long)ny * nz) >> logB);
        k_fft_pass<true, true, false, false>
            <<<grid, threads_of(logN, logB), lds_of(logN, logB), s>>>(
                in, nullptr, nullptr, work, logN, logB, m, twx, +1, 1.f, none);
    }
    // pass 2: y forward
    {
        const int logN = ilog2(ny), logB = pick_B(ny, (long)nx * nz, true);
        LineMap m{nx, ilog2(nx), 1, (long)nx * ny};
        const unsigned grid = (unsigned)(((long)nx * nz) >> logB);
        k_fft_pass<false, false, false, false>
            <<<grid, threads_of(logN, logB), lds_of(logN, logB), s>>>(
                nullptr, work, nullptr, work, logN, logB, m, twy, +1, 1.f, none);
    }
    if (forward_only) {
        // pass 3 without the filter: the forward DFT is left in `work`
        const int logN = ilog2(nz), logB = pick_B(nz, (long)nx * ny, true);
        LineMap m{(long)nx * ny, 40, 1, 0};
        const unsigned grid = (unsigned)(((long)nx * ny) >> logB);
        k_fft_pass<false, false, false, false>
            <<<grid, threads_of(logN, logB), lds_of(logN, logB), s>>>(
                nullptr, work, nullptr, work, logN, logB, m, twz, +1, 1.f, none);
        return hipGetLastError();
    }
    // pass 3: z forward, * H, z inverse
    {
        const int logN = ilog2(nz), logB = pick_B(nz, (long)nx * ny, true);
        LineMap m{(long)nx * ny, 40, 1, 0};
        const unsigned grid = (unsigned)(((long)nx * ny) >> logB);
        k_fft_pass<false, false, false, true>
            <<<grid, threads_of(logN, logB), lds_of(logN, logB), s>>>(
                nullptr, work, nullptr, work, logN, logB, m, twz, +1, 1.f, R);
    }
    // pass 4: y inverse
    {
        const int logN = ilog2(ny), logB = pick_B(ny, (long)nx * nz, true);
        LineMap m{nx, ilog2(nx), 1, (long)nx * ny};
        const unsigned grid = (unsigned)(((long)nx * nz) >> logB);
        k_fft_pass<false, false, false, false>
            <<<grid, threads_of(logN, logB), lds_of(logN, logB), s>>>(
                nullptr, work, nullptr, work, logN, logB, m, twy, -1, 1.f, none);
    }
    // pass 5: x inverse -> real, scaled
    {
        const int logN = ilog2(nx), logB = pick_B(nx, (long)ny * nz, false);
        LineMap m{1, 40, nx, 0};
        const unsigned grid = (unsigned)(((long)ny * nz) >> logB);
        k_fft_pass<true, false, true, false>
            <<<grid, threads_of(logN, logB), lds_of(logN, logB), s>>>(
                nullptr, work, out, nullptr, logN, logB, m, twx, -1, (float)(1.0 / (double)nvox), none);
    }
    return hipGetLastError();
}

// T[k] = Re(X[k] e^{+2 pi i k.c / n}) with X the forward DFT of an impulse
// response centred at voxel c (phase in FP64).
__global__ void k_spectrum_real(const float2 *__restrict__ X, float *__restrict__ T, int nx, int ny, int nz,
                                int cx, int cy, int cz) {
    const long n = (long)nx * ny * nz;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const int kx = (int)(i % nx), ky = (int)((i / nx) % ny), kz = (int)(i / ((long)nx * ny));
        const double ph = 2.0 * M_PI * ((double)((long)kx * cx % nx) / nx + (double)((long)ky * cy % ny) / ny +
                                        (double)((long)kz * cz % nz) / nz);
        const float2 x = X[i];
        T[i] = (float)((double)x.x * cos(ph) - (double)x.y * sin(ph));
    }
}

// H = 1 / max(T, floor_rel * T[0])
__global__ void k_transfer_inverse(const float *T, float *H, long n, double floor_rel) {
    const double fl = floor_rel * (double)T[0];
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        H[i] = (float)(1.0 / fmax((double)T[i], fl));
}

// Shell sums of T by the nearest rho sample (rho as radial_gain computes it),
// in 64-bit fixed point so that the atomics' order does not matter.
__global__ void k_radial_bin(const float *__restrict__ T, int nx, int ny, int nz, int n_table, float rho_max,
                             double scale, unsigned long long *sums, unsigned *counts) {
    const long n = (long)nx * ny * nz;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const int ex = (int)(i % nx), ey = (int)((i / nx) % ny), ez = (int)(i / ((long)nx * ny));
        const int kx = ex < nx / 2 ? ex : ex - nx;
        const int ky = ey < ny / 2 ? ey : ey - ny;
        const int kz = ez < nz / 2 ? ez : ez - nz;
        const float fx = (float)kx / nx, fy = (float)ky / ny, fz = (float)kz / nz;
        const float rho = 2.f * sqrtf(fx * fx + fy * fy + fz * fz);
        const float t = rho / rho_max * (float)(n_table - 1);
        const int b = (int)(t + 0.5f);
        if (b >= n_table) continue;
        const long long q = llrint((double)T[i] * scale);
        atomicAdd(sums + b, (unsigned long long)q);
        atomicAdd(counts + b, 1u);
    }
}

hipError_t launch_spectrum_real(const float2 *X, float *T, int nx, int ny, int nz, hipStream_t s) {
    const long n = (long)nx * ny * nz;
    const unsigned g = (unsigned)std::min<long>((n + 255) / 256, 65535);
    k_spectrum_real<<<g, 256, 0, s>>>(X, T, nx, ny, nz, nx / 2, ny / 2, nz / 2);
    return hipGetLastError();
}
hipError_t launch_transfer_inverse(const float *T, float *H, long n, double floor_rel, hipStream_t s) {
    const unsigned g = (unsigned)std::min<long>((n + 255) / 256, 65535);
    k_transfer_inverse<<<g, 256, 0, s>>>(T, H, n, floor_rel);
    return hipGetLastError();
}
hipError_t launch_radial_bin(const float *T, int nx, int ny, int nz, int n_table, float rho_max, double scale,
                             unsigned long long *sums, unsigned *counts, hipStream_t s) {
    const long n = (long)nx * ny * nz;
    const unsigned g = (unsigned)std::min<long>((n + 255) / 256, 65535);
    k_radial_bin<<<g, 256, 0, s>>>(T, nx, ny, nz, n_table, rho_max, scale, sums, counts);
    return hipGetLastError();
}

}  // namespace mgct
