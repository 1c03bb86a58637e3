/*
 * mgct — preconditioned multigrid Landweber reconstruction for cone-beam CT
 * on AMD Instinct MI355X (gfx950).  C ABI.
 *
 * Method: Myers et al., "Rapidly-converging multigrid reconstruction of
 * cone-beam tomographic data" (arXiv 2103.10329).  Data model: Beer-Lambert,
 * b = ln(I0/I) = P mu (Sec. 2, eq. 1).  Iterations: Landweber / SIRT (eq. 2),
 * preconditioned Landweber (eq. 4, with the 3^3 kernel of eq. 5 or an
 * isotropic Fourier-space deconvolution filter, Sec. 3), OS-EMTR (eq. 3),
 * and the recursive multigrid of Algorithm 1.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every call returns an int status: MGCT_OK (0) or a negative mgct_status.
 *   mgct_status_string() describes a code.  On error nothing is launched.
 * - Buffers: every array argument named "device" is device memory owned by
 *   the caller (the library never frees it).  Arrays named "host" are host
 *   memory, read (or written) before the call returns.
 * - Stream ordering: work is enqueued on `stream` (0 = the null stream); the
 *   outputs are valid once the stream has been synchronised.  Calls that
 *   return a host scalar (residual norms, step sizes, histories) synchronise
 *   the stream themselves.  Outputs are overwritten, never accumulated
 *   (except mgct_prolong_add, whose purpose is to add).
 * - Layouts: a volume is [nz][ny][nx] with x fastest; a detector stack is
 *   [n_views][nv][nu] with u (detector column) fastest.  Geometry is in
 *   physical units; voxel (i,j,k) is centred at
 *   origin + ((i,j,k) - (n-1)/2) * voxel, and pixel (a,b) of view v at
 *   d + (a-(nu-1)/2) u + (b-(nv-1)/2) v.
 * - Grid levels: level g (0 = finest) halves every volume and detector size
 *   g times and doubles the voxel size and the pixel steps g times, with the
 *   same source and detector-centre positions (Algorithm 1 shares the
 *   trajectory between grids).  Sizes must be divisible by 2^g.
 * - A context serialises nothing: calls on one context must not overlap in
 *   time on different streams (they share workspace).
 */
#ifndef MGCT_H
#define MGCT_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MGCT_OK = 0,
    MGCT_ERR_INVALID_ARG = -1,          /* null pointer, bad size, bad enum value */
    MGCT_ERR_UNSUPPORTED_GEOMETRY = -2, /* a ray whose largest direction component is along z */
    MGCT_ERR_SIZE_NOT_DIVISIBLE = -3,   /* a size not divisible by 2^level */
    MGCT_ERR_OOM = -4,                  /* device allocation failed */
    MGCT_ERR_HIP = -5,                  /* a HIP runtime call failed */
    MGCT_ERR_DIVERGED = -6,             /* the residual grew or is not finite: step size too large */
    MGCT_ERR_NOT_IMPLEMENTED = -7,      /* combination not provided (e.g. radial filter on non-power-of-2 grid) */
    MGCT_ERR_NO_GEOMETRY = -8,          /* mgct_set_geometry has not been called */
    MGCT_ERR_TOO_LARGE = -9             /* the grid exceeds mgct_project_noalloc's fixed scratch */
} mgct_status;

typedef enum { MGCT_F32 = 0, MGCT_F16 = 1, MGCT_BF16 = 2 } mgct_dtype;

typedef enum {
    MGCT_FILTER_IDENTITY = 0,  /* p = delta: plain Landweber / SIRT, eq. 2 */
    MGCT_FILTER_STENCIL27 = 1, /* circular 3^3 convolution, eq. 5 taps (or any 27 taps) */
    MGCT_FILTER_RADIAL = 2,    /* circular convolution applied in Fourier space: H(rho) */
    MGCT_FILTER_TRANSFER = 3   /* circular convolution applied in Fourier space: H(k) per grid */
} mgct_filter_kind;

/*
 * Preconditioning kernel p of eq. 4.
 * STENCIL27: taps[(dz+1)*9 + (dy+1)*3 + (dx+1)]; out[z,y,x] = sum taps[d] in[(z,y,x)-d],
 *   indices wrapped (circular).  mgct_filter_eq5() fills in eq. 5.
 * RADIAL: the 3-D DFT of the volume (sized to the grid, circular) is
 *   multiplied by H(rho), rho = 2 sqrt(sum_a (k_a/N_a)^2) with signed
 *   frequencies k_a in [-N_a/2, N_a/2), and H is linear interpolation of
 *   `radial_table` (host, n_table >= 2 samples uniformly on [0, rho_max],
 *   clamped beyond).  Every grid edge must be a power of two, 2..1024.
 * TRANSFER: as RADIAL with an arbitrary real transfer function: the DFT is
 *   multiplied by transfer[level][(kz*ny + ky)*nx + kx] (device F32 array of
 *   the grid's size, unsigned frequency indices as the DFT orders them), one
 *   array per grid the filter is used on (see mgct_psf_spectrum for the one
 *   derived from the scan).  The caller owns the arrays.
 */
typedef struct {
    int kind;
    float taps[27];
    const float *radial_table;
    int n_table;
    float rho_max;
    const float *transfer[8];
} mgct_filter;

/* Parameters of Algorithm 1 (mgct_multigrid_solve). */
typedef struct {
    int levels;            /* L >= 1; grid L-1 is solved by OS-EMTR when L >= 2 */
    int n_outer;           /* full multigrid iterations */
    mgct_filter filter;    /* preconditioner on every Landweber grid */
    double alpha[8];       /* step of grid g (g < L-1, or g = 0 when L = 1); <= 0: 1/lambda_max */
    int power_iters;       /* power iterations for automatic steps (e.g. 30) */
    uint64_t power_seed;   /* SplitMix64 seed of the power-iteration start vector */
    double lambda;         /* soft threshold (0 = off) */
    int bilateral_on;      /* bilateral filter after every Landweber step */
    double sigma_s;        /* spatial sigma, voxels */
    double sigma_r;        /* range sigma, attenuation units */
    int coarse_subsets;    /* OS-EMTR subsets M (views i with i mod M == m) */
    int coarse_passes;     /* OS-EMTR passes over all subsets per coarse solve */
    int learned;           /* finest grid: mu + u + f(u) (the context's network, see
                              mgct_cnn_*), kept only if it lowers ||b - A mu||, else mu + u */
    float *capture_update; /* device, finest-grid volume or NULL: receives the finest grid's
                              filtered update u = alpha p * A^T (b - A mu) of the last iteration */
    float *capture_iterate;/* device, finest-grid volume or NULL: mu just before that update */
} mgct_mg_params;

const char *mgct_status_string(int status);

/* Fill `f` with eq. 5's kernel (taps /64, the printed matrices as z-slices). */
int mgct_filter_eq5(mgct_filter *f);

/* Create a context on HIP device `device` (made current by every call). */
int mgct_create(int device, void **ctx_out);
int mgct_destroy(void *ctx);

/*
 * Geometry of the scan (paper Sec. 2, eq. 1: the projection operator is set
 * by the volume grid and the source/detector positions Theta).
 * views: host, n_views x 12 doubles per view: s[3], d[3], u[3], v[3].
 * The library copies what it needs.  Rejects (UNSUPPORTED_GEOMETRY) any
 * geometry with a ray whose largest |direction component| is along z, and
 * any geometry whose source lies within one voxel of the volume box.
 * Synchronises the device.  A new grid shape (nx, ny, nz) releases the
 * context's device workspaces; the same shape with other views keeps them.
 */
int mgct_set_geometry(void *ctx, int nx, int ny, int nz, double voxel, const double origin[3],
                      int nu, int nv, int n_views, const double *views);

/*
 * proj = A vol on grid `level` (Sec. 2, eq. 1's P): Joseph's method — every
 * ray is sampled on the voxel-centre planes of its major axis between source
 * and pixel, with bilinear interpolation (zero outside the grid), times the
 * sample spacing.  vol: device, vol_dtype F32 or BF16.  proj: device,
 * proj_dtype F32 or F16.  Accumulation is FP32.  A BF16 volume is read as
 * BF16 (the projector's internal copy keeps BF16).
 */
int mgct_project(void *ctx, int level, const void *vol, int vol_dtype, void *proj, int proj_dtype,
                 hipStream_t stream);

/*
 * vol = A^T proj on grid `level` (Sec. 2.1: B is the adjoint of P): exact
 * transpose of mgct_project, evaluated voxel by voxel (a gather; no atomics,
 * so results are bit-identical from run to run).  proj: device, F32 or F16;
 * vol: device, F32 or BF16.  FP32 accumulation per view, FP64 across views.
 * F16 data are pre-scaled into an F16 copy.
 */
int mgct_backproject(void *ctx, int level, const void *proj, int proj_dtype, void *vol, int vol_dtype,
                     hipStream_t stream);

/*
 * Which forward projector the separable geometry (detector columns
 * horizontal, rows vertical) uses when all views are projected at once; both
 * compute the same Joseph sums and return bit-identical results:
 * MGCT_PROJECTOR_GATHER reads each sample's four taps with one 16-byte gather
 * from two pair-expanded volume copies (fast while the copies stay in the
 * caches); MGCT_PROJECTOR_STAGED stages, for a tile of 8 detector columns x
 * 64 rows of one view, the volume window its rays cross into LDS, 8 planes
 * at a time, from one plain copy, with the views ordered so that a band of
 * the volume is shared in the last-level cache; MGCT_PROJECTOR_AUTO (the
 * default) takes the staged one for grids of 256^3 voxels or more.  Other
 * geometries and view subsets always use their own kernels.  Host only.
 */
typedef enum { MGCT_PROJECTOR_AUTO = 0, MGCT_PROJECTOR_GATHER = 1, MGCT_PROJECTOR_STAGED = 2 } mgct_projector;
int mgct_set_projector(void *ctx, int variant);

/*
 * Storage precision of the copies a Landweber step makes (mgct_landweber_step,
 * and every Landweber grid of mgct_multigrid_solve): the projector's copy of
 * the volume (F32 or BF16) and the projected / residual / scaled data stacks
 * (F32 or F16).  Interpolation and accumulation along rays and across views
 * stay FP32 (norms FP64); the OS-EMTR coarse solve, the Fourier filter, the
 * step-size estimate and the iterate itself stay FP32.  Default F32, F32.
 */
int mgct_set_precision(void *ctx, int volume_copy_dtype, int stack_dtype);

/* out = p * in on grid `level` (eq. 4's convolution).  in, out: device F32 volumes (may alias). */
int mgct_precondition(void *ctx, int level, const float *in, float *out, const mgct_filter *f,
                      hipStream_t stream);

/*
 * Step size for eq. 2 / eq. 4 on grid `level`: alpha = 1/lambda with lambda
 * the largest eigenvalue of x -> p * A^T A x, from `iters` power iterations
 * started at SplitMix64 uniforms (output k: state seed + (k+1) * golden
 * gamma).  alpha: host, written.  f may be NULL (identity).
 */
int mgct_estimate_step(void *ctx, int level, const mgct_filter *f, int iters, uint64_t seed,
                       double *alpha, hipStream_t stream);

/*
 * One Landweber step on grid `level`: vol += alpha * p * A^T (b - A vol)
 * (eq. 4; f NULL or IDENTITY gives SIRT, eq. 2).  vol: device F32, updated in
 * place.  b: device stack of that grid, F32 or F16.  resid_norm: host, may be
 * NULL; receives ||b - A vol|| of the input volume (FP64 reduction) and then
 * synchronises the stream.
 * Divergence (Sec. 2.1, eq. 2's step alpha): p is positive semi-definite, so
 * for alpha <= 2/lambda_max(p A^T A) the residual cannot grow from one step to
 * the next, on consistent or inconsistent data.  With resid_norm given, the
 * call returns MGCT_ERR_DIVERGED (after the step has been applied) when the
 * residual is not finite, or when it exceeds the previous call's on the same
 * grid, data pointer, alpha and filter by more than the context's ratio
 * (mgct_set_divergence, default 1.05): alpha exceeds 2/lambda_max.
 */
int mgct_landweber_step(void *ctx, int level, float *vol, const void *b, int b_dtype, double alpha,
                        const mgct_filter *f, double *resid_norm, hipStream_t stream);

/*
 * Ratio of the divergence test of mgct_landweber_step and
 * mgct_multigrid_solve: >= 1, or 0 to report only non-finite residuals.
 * Resets the Landweber steps' residual history.  Host only.
 */
int mgct_set_divergence(void *ctx, double ratio);

/*
 * The divergence rule itself (host only, no device access): 1 when cur is not
 * finite, or when ratio > 0, prev > 0 and cur > ratio * prev; else 0.
 */
int mgct_residual_diverged(double prev, double cur, double ratio);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * projection as mgct_project on grid `level`, with the projector's padded
 * volume copies in a fixed scratch of 40 MiB per GPU (FP32 grids up to about
 * 128^3, BF16 up to about 160^3) instead of context workspaces.  Calls no
 * allocating routine.  The grid's tables must exist: level 0 always does
 * after mgct_set_geometry, another level after any earlier call on it (else
 * MGCT_ERR_INVALID_ARG).  A grid whose copies exceed the scratch returns
 * MGCT_ERR_TOO_LARGE before any launch.  vol, proj, dtypes and the stream as
 * in mgct_project.  Every call on one GPU shares that GPU's scratch (it is
 * cleared where it must start at zero on every call): calls that overlap on
 * one GPU, from any context or stream, race.  No kernel timing is recorded.
 */
int mgct_project_noalloc(void *ctx, int level, const void *vol, int vol_dtype, void *proj, int proj_dtype,
                         hipStream_t stream);

/*
 * Geometry derivative for joint model estimation (paper Sec. 1: geometry
 * such as thermal drift estimated jointly with the image): with the volume
 * vol (device F32, grid `level`) and a cotangent stack cot (device F32,
 * e.g. the residual A vol - b for the gradient of 0.5 ||A vol - b||^2),
 * dviews (host, n_views x 12 doubles, written) receives
 * d/d(view) sum_rays cot * (A vol) for each view's s, d, u, v (physical
 * units), differentiating the Joseph sums with their major axes and plane
 * sets held fixed (the sum is piecewise smooth).  Synchronises the stream.
 * Returns MGCT_ERR_NOT_IMPLEMENTED when the grid's padded FP32 copy would
 * exceed 4 GiB (about 1020^3 voxels).
 */
int mgct_project_geom_grad(void *ctx, int level, const float *vol, const float *cot, double *dviews,
                           hipStream_t stream);

/*
 * Chain rule from per-view gradients (dviews, n_views x 12, host) to the
 * three parameters of a rigid misalignment of every view of views0 (host,
 * n_views x 12, the unperturbed table): dx and dz move the source by
 * dx*voxel along the view's unit column direction and dz*voxel along z; the
 * detector's column and row steps rotate by tilt_deg (degrees) about its
 * normal.  grad (host, 3) = d/d(dx, dz, tilt_deg) at (dx, dz, tilt_deg).
 * Host-only arithmetic.
 */
int mgct_geometry_param_grad(int n_views, const double *views0, const double *dviews, double voxel, double dx,
                             double dz, double tilt_deg, double grad[3]);

/*
 * Derived preconditioners (Sec. 3 leaves more rigorously derived kernels to
 * later work; this measures the one the scan implies).  T = the transfer
 * function of A^T A on grid `level`: the real part of the 3-D DFT of
 * A^T A applied to a unit impulse at voxel (nx/2, ny/2, nz/2), phase-shifted
 * to the origin (A^T A is symmetric, so the spectrum of its impulse
 * response is real up to rounding).  T: device F32 [nz][ny][nx], DFT order.
 * Every grid edge must be a power of two, 2..1024.
 */
int mgct_psf_spectrum(void *ctx, int level, float *T, hipStream_t stream);

/*
 * H = 1 / max(T, floor_rel * T[0]) elementwise (T[0] = the DC gain): the
 * approximate deconvolution of the measured point-spread function, bounded
 * where the scan transmits little.  T, H: device F32 arrays of grid `level`
 * (must not alias: every element reads T[0]; INVALID_ARG if T == H).
 */
int mgct_transfer_from_spectrum(void *ctx, int level, const float *T, double floor_rel, float *H,
                                hipStream_t stream);

/*
 * Shell averages of a spectrum on grid `level`: profile[i] (host, n_table
 * doubles) = mean of T over the frequencies whose rho (as for RADIAL) rounds
 * to sample i of n_table samples on [0, rho_max]; counts (host, may be NULL)
 * receives the number in each shell (0: profile NaN).  Sums are accumulated in
 * 64-bit fixed point (2^-24 units), so the result does not depend on
 * scheduling.  Synchronises the stream.
 */
int mgct_radial_profile(void *ctx, int level, const float *T, int n_table, double rho_max, double *profile,
                        int *counts, hipStream_t stream);

/* Restrict (Algorithm 1): coarse = 2x2x2 block mean of fine (grid level -> level+1). */
int mgct_restrict_volume(void *ctx, int level, const float *fine, float *coarse, hipStream_t stream);

/* Restrict (Algorithm 1) of the data: coarse stack = 2x2 pixel mean of b (grid level -> level+1). */
int mgct_restrict_stack(void *ctx, int level, const float *fine, float *coarse, hipStream_t stream);

/*
 * Prolongate and correct (Algorithm 1): fine += P(coarse_new - coarse_old),
 * P cell-centred trilinear (weights 3/4, 1/4; edges clamped).  fine on grid
 * `level`, coarse arrays on grid level+1.
 */
int mgct_prolong_add(void *ctx, int level, const float *coarse_new, const float *coarse_old, float *fine,
                     hipStream_t stream);

/* SoftThreshold (Algorithm 1): vol = sign(vol) max(|vol| - lambda, 0), in place. */
int mgct_soft_threshold(void *ctx, int level, float *vol, double lambda, hipStream_t stream);

/*
 * BilateralFilter (Algorithm 1): out = normalised 3^3 bilateral filter of in
 * (spatial weight exp(-|d|^2/2 sigma_s^2), range weight
 * exp(-(in_n - in)^2 / 2 sigma_r^2), neighbours outside the grid left out).
 * in and out must not alias.
 */
int mgct_bilateral(void *ctx, int level, const float *in, float *out, double sigma_s, double sigma_r,
                   hipStream_t stream);

/*
 * OS-EMTR (eq. 3) on grid `level`: `passes` passes over M = `subsets`
 * interleaved view subsets; per subset
 * vol += A_m^T(e - exp(-b)) / A_m^T(e * A1), e = exp(-A_m vol),
 * where A1 is A applied to a volume of ones (support = the grid); voxels with
 * denominator <= 1e-6 * max(denominator) are left unchanged.
 * vol: device F32, in place; b: device F32 stack of that grid.
 */
int mgct_osemtr(void *ctx, int level, float *vol, const float *b, int subsets, int passes, hipStream_t stream);

/*
 * Algorithm 1, `p->n_outer` full iterations starting from vol (device F32,
 * in place, finest grid).  b: device stack of the finest grid (F32 or F16).
 * resid_hist: host, may be NULL, n_outer x levels doubles: entry [n][g] is
 * ||b_g - A_g mu|| before grid g's Landweber step (g < L-1) and, for
 * g = L-1, before the coarse OS-EMTR solve.  With resid_hist given the
 * call synchronises the stream and returns MGCT_ERR_DIVERGED (after all
 * iterations) when a recorded residual is not finite or the finest grid's
 * grows between consecutive outer iterations by more than the divergence
 * ratio (mgct_set_divergence).  Automatic step sizes are cached per grid
 * and filter; a TRANSFER filter is identified by its array's contents.
 */
int mgct_multigrid_solve(void *ctx, float *vol, const void *b, int b_dtype, const mgct_mg_params *p,
                         double *resid_hist, hipStream_t stream);

/*
 * Learned preconditioner (an extension beyond the paper's fixed filters; refines eq. 4's filtered
 * update u): out = u + f(u), f = four 3^3 convolutions 1 -> 16 -> 32 -> 32 -> 1
 * with zero "same" padding and erf-GELU after the first three.  Parameters:
 * one FP32 vector of MGCT_CNN_PARAMS values, W1 b1 W2 b2 W3 b3 W4 b4, each W
 * as [out][in][kz][ky][kx] (cross-correlation, as torch's conv3d).  The
 * library keeps an FP32 master copy and Adam state per context; the matrix
 * core layers use BF16 weights and activations with FP32 accumulation.
 * Volumes: device F32 [nz][ny][nx], nx a multiple of 32.
 */
#define MGCT_CNN_PARAMS 42849
int mgct_cnn_set_weights(void *ctx, const float *weights /* host */, int n);  /* also resets Adam */
int mgct_cnn_get_weights(void *ctx, float *weights /* host */, int n);
int mgct_cnn_forward(void *ctx, int nx, int ny, int nz, const float *u, float *out, hipStream_t stream);
/* forward + backward of the mean squared error against target; grads host (n params), loss host (may be NULL) */
int mgct_cnn_gradients(void *ctx, int nx, int ny, int nz, const float *u, const float *target, float *grads,
                       double *loss, hipStream_t stream);
/* forward + backward + one Adam step (beta 0.9/0.999, eps 1e-8) of learning rate lr */
int mgct_cnn_train_step(void *ctx, int nx, int ny, int nz, const float *u, const float *target, double lr,
                        double *loss, hipStream_t stream);
/*
 * The network's backward pass for a loss the caller defines: grads (host,
 * MGCT_CNN_PARAMS values, in the weight vector's layout) = the gradient of
 * sum over voxels of dout * out with respect to the parameters, at input u
 * (device F32 [nz][ny][nx]); dout (device F32, same shape) is d loss / d out.
 * The activations of u are recomputed first.  Synchronises the stream.
 */
int mgct_cnn_backward(void *ctx, int nx, int ny, int nz, const float *u, const float *dout, float *grads,
                      hipStream_t stream);
/*
 * One Adam step (Kingma & Ba, beta 0.9/0.999, eps 1e-8, bias-corrected;
 * the same update as mgct_cnn_train_step's) of learning rate lr on the
 * context's master weights with caller-supplied gradients (host,
 * n = MGCT_CNN_PARAMS values); advances the context's Adam state and
 * re-derives the BF16 operands.  MGCT_ERR_INVALID_ARG without weights set.
 * Synchronises the stream.
 */
int mgct_adam_step(void *ctx, const float *grads, int n, double lr, hipStream_t stream);

/*
 * Learned-step statistics since the last call: finest-grid steps whose
 * network update was kept (accepted) and steps that fell back to the plain
 * filtered update (rejected).  Synchronises the device.
 */
int mgct_learned_stats(void *ctx, int *accepted, int *rejected);

/*
 * The two squared residual norms the learned step's judge compared last:
 * r0 = ||b - A mu||^2 before the finest-grid update, r1 = ||b - A (mu + f(u))||^2
 * with the network's refinement f(u); the refinement was kept iff r1 < r0.
 * On scans of 720 views or more with the staged projector both run over every
 * view_step-th view (view_step = n_views / 360; about 360 views, which spares
 * the judge a full projection), otherwise over all views (view_step 1).
 * Host pointers (view_step may be NULL).  MGCT_ERR_INVALID_ARG before any
 * learned step.  Synchronises the device.
 */
int mgct_learned_judge(void *ctx, double *r0, double *r1, int *view_step);

/*
 * Synthetic data on the device (training-set generation for the learned
 * preconditioner): exact line integrals through a phantom of K ellipsoids and
 * J axis-aligned boxes for every ray of the finest grid's geometry, and the
 * ss^3-supersampled voxel average of the same phantom on the finest grid.
 * Ellipsoid record: centre[3], rotation[9] (row-major, columns = body axes),
 * semi-axes[3], attenuation; box record: lo[3], hi[3], attenuation (host
 * arrays, physical units).  out/vol: device F32, overwritten.
 */
int mgct_synth_line_integrals(void *ctx, const double *ellipsoids, int K, const double *boxes, int J, float *out,
                              hipStream_t stream);
int mgct_synth_voxelize(void *ctx, const double *ellipsoids, int K, const double *boxes, int J, int ss, float *vol,
                        hipStream_t stream);

/*
 * Kernel timing (instrumentation).  While enabled, every launch of the
 * kernels below is bracketed by HIP events recorded on the launch's stream.
 * mgct_kernel_timing(ctx, 1) enables and clears the records, (ctx, 0)
 * disables (records are kept).  mgct_kernel_time() synchronises on the
 * recorded events and returns the summed duration (ms, host) and the number
 * of launches of kernel `op` on grid `level` (level -1: all grids).
 */
typedef enum {
    MGCT_OP_PROJECT = 0,          /* ray-driven projector kernel */
    MGCT_OP_BACKPROJECT = 1,      /* voxel-driven transpose kernel */
    MGCT_OP_PRECONDITION = 2,     /* stencil or Fourier filter (all passes) */
    MGCT_OP_VOLUME_TRANSPOSE = 3, /* volume copy into the projector's layout */
    MGCT_OP_DATA_PRESCALE = 4,    /* data scaling/transposition before A^T */
    MGCT_OP_COUNT = 5
} mgct_op;

int mgct_kernel_timing(void *ctx, int enable);
int mgct_kernel_time(void *ctx, int op, int level, double *total_ms, int *launches);
/*
 * Narrows what is recorded while timing is enabled: a launch of operation op
 * on grid g is bracketed only if bit op of op_mask and bit g of level_mask are
 * set.  A new context records everything (both masks ~0u).  Fewer records keep
 * the events' own cost (each is a command on the stream) out of a timed
 * region.  The masks stay until changed; existing records are kept.
 * MGCT_ERR_INVALID_ARG for a null ctx.
 */
int mgct_kernel_timing_select(void *ctx, unsigned op_mask, unsigned level_mask);

#ifdef __cplusplus
}
#endif

#endif /* MGCT_H */
