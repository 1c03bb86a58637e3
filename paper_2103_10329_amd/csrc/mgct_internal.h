// Internal declarations shared by the host driver and the HIP kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "mgct.h"

namespace mgct {

// Per-view geometry in voxel-index coordinates of one grid level: a point P
// (physical) maps to (P - origin)/h + (n-1)/2, so voxel (i,j,k) sits at
// integer coordinates (i,j,k).  Vectors scale by 1/h.
struct ViewIdx {
    double s[3], d[3], u[3], v[3];
};

// Per-view constants of the separable back-projector (geometry with the
// detector columns horizontal and the rows along z): the ray of pixel (a,b)
// has direction (Dx(a), Dy(a), dz0 + b*vz); the detector column hit by the
// ray through (px, py, .) is (an0 + an1 px + an2 py)/(ad0 + ad1 px + ad2 py).
struct SepView {
    double sx, sy, sz, dz0, vz;
    double r0lo, r0hi;  // range of 1/Dx over the view's x-major columns
    double r1lo, r1hi;  // range of 1/Dy over its y-major columns
    float an0, an1, an2, ad0, ad1, ad2;
    int flags;  // bit 0: the view has x-major columns, bit 1: y-major columns
    int pad;
};

// Per-(view, column) ray direction of the separable geometry.
// 64 bytes: one scalar load per column.
struct ColD {
    double dx, dy, rdx, rdy;  // Dx(a), Dy(a), 1/Dx(a), 1/Dy(a)
    double dxv, dyv;          // Dx(a)/vz, Dy(a)/vz
    int axis;                 // 0: x-major, 1: y-major
    int pad[3];
};

// Padding (voxels) around the transposed volume copy read by the projector.
constexpr int kVolPad = 2;
// Bytes allocated past the end of the plain padded copy: the LDS projector
// stages whole 64-value z runs and may read up to 63 values past a run's end.
constexpr size_t kCopyTail = 256;

struct Level {
    int nx = 0, ny = 0, nz = 0, nu = 0, nv = 0, nviews = 0;
    double h = 0.0;
    bool separable = false;
    // device tables
    ViewIdx *d_views = nullptr;      // [view]
    SepView *d_sep = nullptr;        // [view]       (separable only)
    ColD *d_cols = nullptr;          // [view][nu] (separable only)
    uint8_t *d_axis = nullptr;       // [view][nu] (separable) or [view][nv][nu]: 0 = x, 1 = y
    int *d_order = nullptr;          // (separable) LDS projector's (view, row tile) order, view * n_rt + tile
    int n_rt = 0;                    // row tiles of 64 rows
    // the learned step's judge views (every judge_step-th view; judge_step 1: all views) as a sub-list of
    // d_order, n_t_judge entries (null when judge_step is 1)
    int judge_step = 1, n_t_judge = 0;
    int *d_order_judge = nullptr;
    long axis_row_stride = 0;        // 0 (separable) or nu
    size_t vox() const { return (size_t)nx * ny * nz; }
    size_t rays() const { return (size_t)nviews * nu * nv; }
    size_t padded_vox() const {
        return (size_t)(nx + 2 * kVolPad) * (ny + 2 * kVolPad) * (nz + 2 * kVolPad);
    }
};

// ---- learned preconditioner (cnn.hip)
constexpr int kCnnParams = 42849;  // 1->16->32->32->1 channels, 3^3 kernels, biases

struct CnnState {
    float *master = nullptr;  // FP32 parameters [W1 b1 W2 b2 W3 b3 W4 b4]
    float *adam_m = nullptr, *adam_v = nullptr, *grads = nullptr;
    uint16_t *p2f = nullptr, *p3f = nullptr, *p3d = nullptr, *p2d = nullptr;  // packed BF16 operands
    uint16_t *p4 = nullptr;  // layer 4's weights as BF16 pairs for the matrix-core kernel
    uint16_t *p1 = nullptr;  // layer 1's weights as three exact BF16 pieces
    int adam_t = 0;
    bool ready = false;
};

// activation / gradient buffers for one volume of n voxels
struct CnnBuffers {
    float *z1 = nullptr, *z2 = nullptr, *z3 = nullptr;      // pre-activations, FP32 [n][C]
    uint16_t *h1 = nullptr, *h2 = nullptr, *h3 = nullptr;   // activations, BF16 [n][C]
    float *dout = nullptr;                                  // [n]
    uint16_t *dz3 = nullptr, *dz2 = nullptr, *dz1 = nullptr;
    uint16_t *gT = nullptr, *xT = nullptr;                  // channels-first copies for weight gradients
    float *partial = nullptr;
    float *up = nullptr;  // the input with a zero border, (nx + 2)(ny + 2)(nz + 2)
};

hipError_t cnn_pack(CnnState &S, hipStream_t s);
hipError_t cnn_forward(CnnState &S, const CnnBuffers &B, const float *u, float *out, int nx, int ny, int nz,
                       bool keep, hipStream_t s);
hipError_t cnn_backward(CnnState &S, const CnnBuffers &B, const float *u, const float *out, const float *target,
                        float *grads, double *loss_partials, int n_loss_blocks, int nx, int ny, int nz,
                        hipStream_t s);
hipError_t cnn_adam(CnnState &S, const float *grads, float lr, hipStream_t s);

struct Ctx {
    int device = 0;
    bool has_geom = false;
    // finest-grid geometry as given
    int nx = 0, ny = 0, nz = 0, nu = 0, nv = 0, nviews = 0;
    double h = 0.0, origin[3] = {0, 0, 0};
    std::vector<double> views;  // n_views x 12
    // grid levels, built on demand; a fixed array so that pointers to a
    // level stay valid while other levels are built
    static constexpr int kMaxLevels = 11;
    Level levels[kMaxLevels];
    // named device workspaces, grown on demand and kept
    std::map<std::string, std::pair<void *, size_t>> ws;
    // cached step sizes keyed by a description of (level, filter, iters, seed)
    std::map<std::string, double> alpha_cache;
    bool pi_valid[kMaxLevels] = {};  // OS-EMTR support projection A 1 cached per level
    // kernel timing records (start/stop events per launch)
    struct TimedLaunch {
        int op, level;
        hipEvent_t start, stop;
    };
    // storage of the Landweber steps' internal copies: the projector's
    // volume copy (F32 or BF16) and the data/residual stacks (F32 or F16)
    int vt_dtype = MGCT_F32, stack_dtype = MGCT_F32;
    int proj_variant = MGCT_PROJECTOR_AUTO;  // mgct_set_projector
    int judge_step_used = 0;                 // view step of the last learned step's judge (0: none yet)
    // divergence status: a Landweber step whose input residual exceeds the
    // previous step's (same grid, data, step size and filter) by more than
    // this factor, or a multigrid solve whose fine-grid residual grows by it
    // between outer iterations, reports MGCT_ERR_DIVERGED; 0 disables
    double diverge_ratio = 1.05;
    struct LwChain {
        bool valid = false;
        const void *b = nullptr;
        double alpha = 0.0, prev = 0.0;
        std::string filter;
    } lw_chain[kMaxLevels];
    CnnState cnn;
    bool timing = false;
    unsigned timing_ops = ~0u, timing_levels = ~0u;  // which (op, grid) pairs are recorded
    std::vector<TimedLaunch> timed;
    std::vector<hipEvent_t> event_pool;
};

// Brackets one kernel launch with events when timing is enabled.
struct KernelTimer {
    Ctx &c;
    int op, level;
    hipStream_t s;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    KernelTimer(Ctx &c_, int op_, int level_, hipStream_t s_);
    ~KernelTimer();
};

// ----- host helpers (api.cpp / geometry.cpp)
int build_level(Ctx &c, int g, Level &out);  // fills host+device tables
void free_level(Level &L);
// (x, y, z) of a linear index i of an [nz][ny][nx] array in 32-bit unsigned
// arithmetic (a 64-bit division costs several times as many instructions);
// every array here holds fewer than 2^32 elements.
__device__ __forceinline__ void split3(size_t i, int nx, int ny, int &x, int &y, int &z) {
    const unsigned u = (unsigned)i, t = u / (unsigned)nx;
    x = (int)(u - t * (unsigned)nx);
    y = (int)(t % (unsigned)ny);
    z = (int)(t / (unsigned)ny);
}

int check_geometry(int nx, int ny, int nz, double h, const double *origin, int nu, int nv, int nviews,
                   const double *views);

// ----- kernel launchers (return hipError_t as int)
// Joseph projector / back-projector (joseph.hip)
hipError_t launch_transpose_volume(const void *vol, int vol_dtype, void *vt, int vt_dtype, const Level &L,
                                   hipStream_t s);
hipError_t launch_project(const void *vt, int vt_dtype, void *proj, int proj_dtype, const Level &L,
                          int view0, int view_step, int nviews_sub, hipStream_t s);
// separable geometry, all views: the LDS-staged projector reading the plain
// padded copy (launch_transpose_volume's layout); mode as for
// launch_project_sep_mode (no OS-EMTR terms); partials: project_lds_blocks().
// order / n_t: another (view, row tile) list than L.d_order (the judge's
// views), whose blocks then fill n_ct x n_t partials.
bool project_lds_ok(const Level &L, int nviews_sub, int variant);
size_t project_lds_blocks(const Level &L);
size_t project_lds_blocks_judge(const Level &L);
hipError_t launch_project_lds_mode(const void *vt, int vt_dtype, int mode, void *out, int out_dtype, const void *y,
                                   int y_dtype, double *partials, const Level &L, hipStream_t s,
                                   const int *order = nullptr, int n_t = -1);
// separable geometry: pair-expanded copies for x-major and y-major rays
size_t pair_copy_elems(const Level &L);
hipError_t launch_transpose_pairs(const void *vol, int vol_dtype, void *vtx, void *vty, int vt_dtype, const Level &L,
                                  hipStream_t s);
hipError_t launch_project_sep(const void *vtx, const void *vty, int vt_dtype, void *proj, int proj_dtype,
                              const Level &L, int view0, int view_step, int nviews_sub, hipStream_t s);
// The separable projector with a fused epilogue (mode: 0 plain, 1 residual
// y - A mu transposed and scaled for A^T plus block partial sums of its
// square, 2 OS-EMTR subset terms, 3 block partial sums of (y - A mu)^2 only);
// partials holds project_sep_blocks() doubles.
hipError_t launch_project_sep_mode(const void *vtx, const void *vty, int vt_dtype, int mode, void *out, void *out2,
                                   int out_dtype, const void *y, int y_dtype, const float *pi, double *partials,
                                   const Level &L, int view0, int view_step, int nviews_sub, hipStream_t s);
size_t project_sep_blocks(const Level &L, int nviews_sub, int vt_dtype);  // vt_dtype: the pair copies' type
// OS-EMTR update that also refreshes the separable projector's pair copies
hipError_t launch_emtr_update_pairs(float *vol, const float *num, const float *den, const unsigned *maxbits,
                                    void *vtx, void *vty, int vt_dtype, const Level &L, hipStream_t s);
hipError_t launch_scale_transpose_stack(const void *proj, int proj_dtype, void *pt, int pt_dtype, const Level &L,
                                        int view0, int view_step, int nviews_sub, hipStream_t s);
// scratch: backproject_scratch_bytes() bytes (partial volumes when the views
// are split over several chunks of waves for small grids), may be null if 0
size_t backproject_scratch_bytes(const Level &L, int nviews_sub, int np);
hipError_t launch_backproject(const void *pt, int pt_dtype, void *vol, int vol_dtype, float *scratch, const Level &L,
                              int view0, int view_step, int nviews_sub, hipStream_t s);
hipError_t launch_backproject2(const float *pt0, const float *pt1, float *vol0, float *vol1, float *scratch,
                               const Level &L, int view0, int view_step, int nviews_sub, hipStream_t s,
                               int *nchunks_left = nullptr);

// general-geometry transpose (any detector orientation; F32 output)
size_t backproject_gen_scratch_bytes(const Level &L, int nviews_sub);
hipError_t launch_backproject_gen(const void *pt, int pt_dtype, float *vol, float *scratch, const Level &L, int view0,
                                  int view_step, int nviews_sub, hipStream_t s);
// derivative with respect to the views' (s, d, u, v); dviews: device, views x 12
size_t geom_grad_partial_bytes(const Level &L);
hipError_t launch_geom_grad(const void *vt, int vt_dtype, const float *cot, double *partial, double *dviews,
                            const Level &L, hipStream_t s);

// Volume / stack operations (volume_ops.hip)
hipError_t launch_fill(float *x, size_t n, float value, hipStream_t s);
hipError_t launch_copy(const float *x, float *y, size_t n, hipStream_t s);
hipError_t launch_convert_to_f32(const void *x, int dtype, float *y, size_t n, hipStream_t s);
hipError_t launch_residual(const void *b, int b_dtype, const void *ax, void *r, int ax_dtype, size_t n,
                           double *partials, int nblocks, hipStream_t s);
hipError_t launch_sumsq(const float *x, size_t n, double *partials, int nblocks, hipStream_t s);
hipError_t launch_finish_sum(const double *partials, int n, double *out, hipStream_t s);
// The same for many partials (two fixed-order stages; tmp holds 256 doubles).
hipError_t launch_finish_sum_wide(const double *partials, int n, double *tmp, double *out, hipStream_t s);
// the sum of the LDS projector's block partials (n_t x n_ct, block t of view
// order[t] / n_rt) over the views with v % step == 0
hipError_t launch_finish_sum_views(const double *partials, const int *order, int n_ct, int n_t, int n_rt, int step,
                                   double *tmp, double *out, hipStream_t s);
hipError_t launch_axpy(float *y, const float *x, double alpha, size_t n, hipStream_t s);
hipError_t launch_scale_by_inv_sqrt(float *x, size_t n, const double *sumsq, double *lambda_out,
                                    hipStream_t s);
hipError_t launch_soft_threshold(float *x, size_t n, float lambda, hipStream_t s);
hipError_t launch_stencil27(const float *in, float *out, int nx, int ny, int nz, const float *taps,
                            hipStream_t s);
hipError_t launch_bilateral(const float *in, float *out, int nx, int ny, int nz, float sigma_s, float sigma_r,
                            hipStream_t s);
hipError_t launch_restrict_volume(const float *fine, float *coarse, int nx, int ny, int nz, hipStream_t s);
hipError_t launch_restrict_stack(const float *fine, float *coarse, int nviews, int nv, int nu, hipStream_t s);
hipError_t launch_prolong_add(const float *cnew, const float *cold, float *fine, int nx, int ny, int nz,
                              hipStream_t s);
hipError_t launch_emtr_update(float *vol, const float *num, const float *den, size_t n, unsigned *maxbits,
                              hipStream_t s);
// OS-EMTR fused steps: subset terms + transposition for A^T; chunk sums + max
hipError_t launch_emtr_terms_t(const float *l, const float *y, const float *pi, float *pt_num, float *pt_den,
                               const Level &L, int view0, int view_step, int nviews_sub, hipStream_t s);
hipError_t launch_emtr_reduce(const float *part_num, const float *part_den, float *num, float *den, size_t n,
                              int nchunks, unsigned *maxbits, hipStream_t s);
hipError_t launch_splitmix_uniform(float *x, size_t n, uint64_t seed, hipStream_t s);
// order-independent 64-bit content key of n_words 32-bit words (partials:
// nblocks values of scratch); out: one device value
hipError_t launch_hash_words(const void *x, size_t n_words, unsigned long long *partials, int nblocks,
                             unsigned long long *out, hipStream_t s);

hipError_t launch_scale(const float *x, float *y, float a, size_t n, hipStream_t s);
hipError_t launch_add(const float *x, const float *y, float *out, size_t n, hipStream_t s);
hipError_t launch_select_update(float *mu, const float *u, const float *mu_try, size_t n, const double *r0,
                                const double *r1, unsigned *counters, hipStream_t s);

// synthetic phantoms on the device (phantom_gpu.hip)
hipError_t launch_synth_line_integrals(const double *views, int nviews, int nu, int nv, const double *ell, int K,
                                       const double *box, int J, float *out, hipStream_t s);
hipError_t launch_synth_voxelize(int nx, int ny, int nz, double h, const double *origin, const double *ell, int K,
                                 const double *box, int J, int ss, float *vol, hipStream_t s);

// FFT preconditioner (fft.hip)
bool fft_size_ok(int n);
hipError_t launch_radial_filter(const float *in, float *out, float2 *work, int nx, int ny, int nz,
                                const float *table, int n_table, float rho_max, const float2 *tw_all, hipStream_t s,
                                const float *hk = nullptr, bool forward_only = false);
// transfer function of an impulse response centred at (nx/2, ny/2, nz/2)
// from its forward DFT; H = 1/max(T, floor T[0]); fixed-point shell sums
hipError_t launch_spectrum_real(const float2 *X, float *T, int nx, int ny, int nz, hipStream_t s);
hipError_t launch_transfer_inverse(const float *T, float *H, long n, double floor_rel, hipStream_t s);
hipError_t launch_radial_bin(const float *T, int nx, int ny, int nz, int n_table, float rho_max, double scale,
                             unsigned long long *sums, unsigned *counts, hipStream_t s);
void host_twiddles(int n, std::vector<float2> &tw);  // exp(-2 pi i k / n), k < n/2

}  // namespace mgct
