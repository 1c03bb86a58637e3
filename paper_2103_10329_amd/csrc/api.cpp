// C-ABI entry points and the host-side orchestration of the iterations
// (Landweber / SIRT, OS-EMTR, power iteration, Algorithm 1).  Every
// arithmetic step runs in the HIP kernels; this file validates arguments,
// manages workspaces and enqueues kernels on the caller's stream.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "mgct_internal.h"

using namespace mgct;

// the fixed scratch of mgct_project_noalloc (end of this file)
static int static_scratch_setup(int device);

#define HIPCHK(x)                                  \
    do {                                           \
        hipError_t e_ = (x);                       \
        if (e_ != hipSuccess) return MGCT_ERR_HIP; \
    } while (0)
#define MGCHK(x)                 \
    do {                         \
        int r_ = (x);            \
        if (r_ != MGCT_OK) return r_; \
    } while (0)

namespace mgct {

static hipEvent_t take_event(Ctx &c) {
    if (!c.event_pool.empty()) {
        hipEvent_t e = c.event_pool.back();
        c.event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

KernelTimer::KernelTimer(Ctx &c_, int op_, int level_, hipStream_t s_) : c(c_), op(op_), level(level_), s(s_) {
    if (!c.timing || op < 0 || op >= 32 || level < 0 || level >= 32) return;
    if (!((c.timing_ops >> op) & 1u) || !((c.timing_levels >> level) & 1u)) return;
    e0 = take_event(c);
    e1 = take_event(c);
    if (e0 && e1) (void)hipEventRecord(e0, s);
}

KernelTimer::~KernelTimer() {
    if (!e0 || !e1) return;
    (void)hipEventRecord(e1, s);
    c.timed.push_back({op, level, e0, e1});
}

}  // namespace mgct

namespace {

constexpr int kRedBlocks = 1024;

Ctx *as_ctx(void *p) { return static_cast<Ctx *>(p); }

void *workspace(Ctx &c, const std::string &name, size_t bytes, bool zero = false) {
    if (bytes == 0) bytes = 1;
    auto it = c.ws.find(name);
    if (it != c.ws.end()) {
        if (it->second.second >= bytes) return it->second.first;
        (void)hipFree(it->second.first);
        c.ws.erase(it);
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    if (zero && hipMemset(p, 0, bytes) != hipSuccess) {
        (void)hipFree(p);
        return nullptr;
    }
    c.ws[name] = {p, bytes};
    return p;
}

#define WS(var, type, name, bytes, zero)                                   \
    type *var = static_cast<type *>(workspace(c, (name), (bytes), (zero))); \
    if (!var) return MGCT_ERR_OOM

int get_level(Ctx &c, int g, Level **out) {
    if (!c.has_geom) return MGCT_ERR_NO_GEOMETRY;
    if (g < 0 || g >= Ctx::kMaxLevels) return MGCT_ERR_INVALID_ARG;
    Level &L = c.levels[g];
    if (L.nx == 0) {
        int r = build_level(c, g, L);
        if (r != MGCT_OK) {
            free_level(L);
            L = Level();
            return r;
        }
    }
    *out = &L;
    return MGCT_OK;
}

std::string lvl(const char *name, int g) { return std::string(name) + "@" + std::to_string(g); }

bool vol_dtype_ok(int d) { return d == MGCT_F32 || d == MGCT_BF16; }
bool stack_dtype_ok(int d) { return d == MGCT_F32 || d == MGCT_F16; }

// ---- projector and transpose on a subset of views (view0 + k*step, k < nsub)
// The separable projector's pair copies of grid g in dtype vt_dtype, filled
// from vol (zero pads survive: allocated zeroed, never written).
int pair_copies(Ctx &c, Level &L, int g, const void *vol, int vol_dtype, int vt_dtype, void **vtx, void **vty,
                hipStream_t s) {
    const bool f32 = vt_dtype == MGCT_F32;
    const size_t es = f32 ? 4 : 2;
    *vtx = workspace(c, lvl(f32 ? "vtx32" : "vtx16", g), pair_copy_elems(L) * es, true);
    *vty = workspace(c, lvl(f32 ? "vty32" : "vty16", g), pair_copy_elems(L) * es, true);
    if (!*vtx || !*vty) return MGCT_ERR_OOM;
    KernelTimer t(c, MGCT_OP_VOLUME_TRANSPOSE, g, s);
    HIPCHK(launch_transpose_pairs(vol, vol_dtype, *vtx, *vty, vt_dtype, L, s));
    return MGCT_OK;
}

// The plain padded z-fastest copy of grid g (zero borders survive: allocated
// zeroed, never written there) read by the LDS projector and the general one.
int plain_copy(Ctx &c, Level &L, int g, const void *vol, int vol_dtype, int vt_dtype, void **vt, hipStream_t s) {
    const size_t es = vt_dtype == MGCT_F32 ? 4 : 2;
    *vt = workspace(c, lvl(vt_dtype == MGCT_F32 ? "vt32" : "vt16", g), L.padded_vox() * es + kCopyTail, true);
    if (!*vt) return MGCT_ERR_OOM;
    KernelTimer t(c, MGCT_OP_VOLUME_TRANSPOSE, g, s);
    HIPCHK(launch_transpose_volume(vol, vol_dtype, *vt, vt_dtype, L, s));
    return MGCT_OK;
}

int do_project(Ctx &c, Level &L, int g, const void *vol, int vol_dtype, void *proj, int proj_dtype, int view0,
               int step, int nsub, hipStream_t s, int vt_dtype = -1) {
    // the projector's volume copy: BF16 when the input is BF16 or when asked
    if (vt_dtype < 0 || vol_dtype == MGCT_BF16) vt_dtype = vol_dtype;
    const size_t es = vt_dtype == MGCT_F32 ? 4 : 2;
    if (L.separable && view0 == 0 && step == 1 && project_lds_ok(L, nsub, c.proj_variant)) {
        void *vt;
        MGCHK(plain_copy(c, L, g, vol, vol_dtype, vt_dtype, &vt, s));
        KernelTimer t(c, MGCT_OP_PROJECT, g, s);
        HIPCHK(launch_project_lds_mode(vt, vt_dtype, 0, proj, proj_dtype, nullptr, MGCT_F32, nullptr, L, s));
        return MGCT_OK;
    }
    if (L.separable) {
        void *vtx, *vty;
        MGCHK(pair_copies(c, L, g, vol, vol_dtype, vt_dtype, &vtx, &vty, s));
        KernelTimer t(c, MGCT_OP_PROJECT, g, s);
        HIPCHK(launch_project_sep(vtx, vty, vt_dtype, proj, proj_dtype, L, view0, step, nsub, s));
        return MGCT_OK;
    }
    void *vt = workspace(c, lvl(vt_dtype == MGCT_F32 ? "vt32" : "vt16", g), L.padded_vox() * es + kCopyTail, true);
    if (!vt) return MGCT_ERR_OOM;
    {
        KernelTimer t(c, MGCT_OP_VOLUME_TRANSPOSE, g, s);
        HIPCHK(launch_transpose_volume(vol, vol_dtype, vt, vt_dtype, L, s));
    }
    KernelTimer t(c, MGCT_OP_PROJECT, g, s);
    HIPCHK(launch_project(vt, vt_dtype, proj, proj_dtype, L, view0, step, nsub, s));
    return MGCT_OK;
}

int do_backproject_pt(Ctx &c, Level &L, int g, const void *pt, int pt_dtype, void *vol, int vol_dtype, int view0,
                      int step, int nsub, hipStream_t s);

int do_backproject(Ctx &c, Level &L, int g, const void *proj, int proj_dtype, void *vol, int vol_dtype, int view0,
                   int step, int nsub, hipStream_t s, int pt_dtype = -1) {
    if (!L.separable && vol_dtype != MGCT_F32) return MGCT_ERR_NOT_IMPLEMENTED;
    // the scaled, transposed data copy: F16 when the input is F16 or when asked
    if (pt_dtype < 0 || proj_dtype == MGCT_F16) pt_dtype = proj_dtype;
    const size_t es = pt_dtype == MGCT_F32 ? 4 : 2;
    WS(pt, char, lvl(pt_dtype == MGCT_F32 ? "pt" : "pt16", g), (size_t)nsub * L.nu * L.nv * es, false);
    {
        KernelTimer t(c, MGCT_OP_DATA_PRESCALE, g, s);
        HIPCHK(launch_scale_transpose_stack(proj, proj_dtype, pt, pt_dtype, L, view0, step, nsub, s));
    }
    return do_backproject_pt(c, L, g, pt, pt_dtype, vol, vol_dtype, view0, step, nsub, s);
}

// A^T from the scaled, transposed copy pt ([view][column][row], ray-length
// factors applied) of a stack.
int do_backproject_pt(Ctx &c, Level &L, int g, const void *pt, int pt_dtype, void *vol, int vol_dtype, int view0,
                      int step, int nsub, hipStream_t s) {
    const size_t sb = L.separable ? backproject_scratch_bytes(L, nsub, 1) : backproject_gen_scratch_bytes(L, nsub);
    float *scratch = nullptr;
    if (sb) {
        scratch = static_cast<float *>(workspace(c, lvl("bp_scratch", g), sb, false));
        if (!scratch) return MGCT_ERR_OOM;
    }
    KernelTimer t(c, MGCT_OP_BACKPROJECT, g, s);
    if (L.separable)
        HIPCHK(launch_backproject(pt, pt_dtype, vol, vol_dtype, scratch, L, view0, step, nsub, s));
    else
        HIPCHK(launch_backproject_gen(pt, pt_dtype, (float *)vol, scratch, L, view0, step, nsub, s));
    return MGCT_OK;
}

int check_filter(const mgct_filter *f, const Level &L, int g) {
    if (!f) return MGCT_OK;
    if (f->kind == MGCT_FILTER_IDENTITY || f->kind == MGCT_FILTER_STENCIL27) return MGCT_OK;
    if (f->kind == MGCT_FILTER_RADIAL || f->kind == MGCT_FILTER_TRANSFER) {
        if (f->kind == MGCT_FILTER_RADIAL && (!f->radial_table || f->n_table < 2 || !(f->rho_max > 0.f)))
            return MGCT_ERR_INVALID_ARG;
        if (f->kind == MGCT_FILTER_TRANSFER && (g < 0 || g >= 8 || !f->transfer[g])) return MGCT_ERR_INVALID_ARG;
        if (!fft_size_ok(L.nx) || !fft_size_ok(L.ny) || !fft_size_ok(L.nz)) return MGCT_ERR_NOT_IMPLEMENTED;
        return MGCT_OK;
    }
    return MGCT_ERR_INVALID_ARG;
}

// Twiddles of grid L's three edges, uploaded once per size.
int fft_twiddles(Ctx &c, const Level &L, float2 **tw_out) {
    const size_t ntw = L.nx / 2 + L.ny / 2 + L.nz / 2;
    std::string twname = "tw_" + std::to_string(L.nx) + "_" + std::to_string(L.ny) + "_" + std::to_string(L.nz);
    bool fresh = c.ws.find(twname) == c.ws.end();
    WS(tw, float2, twname, ntw * sizeof(float2), false);
    if (fresh) {
        std::vector<float2> all, t;
        host_twiddles(L.nx, t);
        all.insert(all.end(), t.begin(), t.begin() + L.nx / 2);
        host_twiddles(L.ny, t);
        all.insert(all.end(), t.begin(), t.begin() + L.ny / 2);
        host_twiddles(L.nz, t);
        all.insert(all.end(), t.begin(), t.begin() + L.nz / 2);
        HIPCHK(hipMemcpy(tw, all.data(), ntw * sizeof(float2), hipMemcpyHostToDevice));
    }
    *tw_out = tw;
    return MGCT_OK;
}

// Device copy of a small host table (filter taps or radial profile), one
// per distinct content: uploaded (synchronously) the first time its bytes are
// seen, reused afterwards, so steady-state filtering issues no host copies.
int device_table(Ctx &c, const char *kind, const float *host, int n, float **dev) {
    uint64_t hsh = 1469598103934665603ull;
    const unsigned char *p = (const unsigned char *)host;
    for (size_t i = 0; i < (size_t)n * 4; ++i) hsh = (hsh ^ p[i]) * 1099511628211ull;
    const std::string key = std::string(kind) + "_" + std::to_string(n) + "_" + std::to_string(hsh);
    const bool fresh = c.ws.find(key) == c.ws.end();
    float *d = static_cast<float *>(workspace(c, key, (size_t)n * 4, false));
    if (!d) return MGCT_ERR_OOM;
    if (fresh) HIPCHK(hipMemcpy(d, host, (size_t)n * 4, hipMemcpyHostToDevice));
    *dev = d;
    return MGCT_OK;
}

int do_precondition(Ctx &c, Level &L, int g, const float *in, float *out, const mgct_filter *f, hipStream_t s) {
    MGCHK(check_filter(f, L, g));
    const size_t n = L.vox();
    if (!f || f->kind == MGCT_FILTER_IDENTITY) {
        if (in != out) HIPCHK(launch_copy(in, out, n, s));
        return MGCT_OK;
    }
    if (f->kind == MGCT_FILTER_STENCIL27) {
        float *taps;
        MGCHK(device_table(c, "taps27", f->taps, 27, &taps));
        KernelTimer t(c, MGCT_OP_PRECONDITION, g, s);
        const float *src = in;
        if (in == out) {
            WS(tmp, float, lvl("st_tmp", g), n * 4, false);
            HIPCHK(launch_copy(in, tmp, n, s));
            src = tmp;
        }
        HIPCHK(launch_stencil27(src, out, L.nx, L.ny, L.nz, taps, s));
        return MGCT_OK;
    }
    // RADIAL or TRANSFER
    float2 *tw;
    MGCHK(fft_twiddles(c, L, &tw));
    WS(work, float2, "fft_work", n * sizeof(float2), false);
    if (f->kind == MGCT_FILTER_TRANSFER) {
        KernelTimer t(c, MGCT_OP_PRECONDITION, g, s);
        HIPCHK(launch_radial_filter(in, out, work, L.nx, L.ny, L.nz, nullptr, 0, 1.f, tw, s, f->transfer[g]));
        return MGCT_OK;
    }
    float *table;
    MGCHK(device_table(c, "radial_table", f->radial_table, f->n_table, &table));
    KernelTimer t(c, MGCT_OP_PRECONDITION, g, s);
    HIPCHK(launch_radial_filter(in, out, work, L.nx, L.ny, L.nz, table, f->n_table, f->rho_max, tw, s));
    return MGCT_OK;
}

// norm2_out: device double receiving ||b - A vol||^2 (may be null).  With
// update_out set, the filtered update alpha p * A^T (b - A vol) is written
// there and vol is left unchanged.
int do_landweber(Ctx &c, Level &L, int g, float *vol, const void *b, int b_dtype, double alpha, const mgct_filter *f,
                 double *norm2_out, hipStream_t s, float *update_out = nullptr) {
    // internal storage per the context's precision setting; arithmetic and
    // accumulation stay FP32 (FP64 for the norm)
    const int sd = c.stack_dtype;
    const size_t es = sd == MGCT_F32 ? 4 : 2;
    if (L.separable) {
        // fused: the projector writes the transposed, scaled residual that
        // A^T reads, and the partial sums of its squared norm
        WS(grad, float, lvl("lw_g", g), L.vox() * 4, false);
        WS(pt, char, lvl(sd == MGCT_F32 ? "pt" : "pt16", g), L.rays() * es, false);
        const int vtd = c.vt_dtype;
        const bool lds = project_lds_ok(L, L.nviews, c.proj_variant);
        const size_t nblk = lds ? project_lds_blocks(L) : project_sep_blocks(L, L.nviews, vtd);
        WS(pp, double, "proj_partials", nblk * 8, false);
        WS(pp2, double, "proj_partials2", 256 * 8, false);
        WS(nrm, double, "red_scratch", 8, false);
        if (lds) {
            void *vt;
            MGCHK(plain_copy(c, L, g, vol, MGCT_F32, vtd, &vt, s));
            KernelTimer t(c, MGCT_OP_PROJECT, g, s);
            HIPCHK(launch_project_lds_mode(vt, vtd, 1, pt, sd, b, b_dtype, pp, L, s));
        } else {
            void *vtx, *vty;
            MGCHK(pair_copies(c, L, g, vol, MGCT_F32, vtd, &vtx, &vty, s));
            KernelTimer t(c, MGCT_OP_PROJECT, g, s);
            HIPCHK(launch_project_sep_mode(vtx, vty, vtd, 1, pt, nullptr, sd, b, b_dtype, nullptr, pp, L, 0, 1,
                                           L.nviews, s));
        }
        HIPCHK(launch_finish_sum_wide(pp, (int)nblk, pp2, norm2_out ? norm2_out : nrm, s));
        MGCHK(do_backproject_pt(c, L, g, pt, sd, grad, MGCT_F32, 0, 1, L.nviews, s));
        MGCHK(do_precondition(c, L, g, grad, grad, f, s));
        if (update_out)
            HIPCHK(launch_scale(grad, update_out, (float)alpha, L.vox(), s));
        else
            HIPCHK(launch_axpy(vol, grad, alpha, L.vox(), s));
        return MGCT_OK;
    }
    WS(ax, char, lvl(sd == MGCT_F32 ? "lw_ax" : "lw_ax16", g), L.rays() * es, false);
    WS(r, char, lvl(sd == MGCT_F32 ? "lw_r" : "lw_r16", g), L.rays() * es, false);
    WS(grad, float, lvl("lw_g", g), L.vox() * 4, false);
    WS(part, double, "red_partials", kRedBlocks * 8, false);
    WS(nrm, double, "red_scratch", 8, false);
    MGCHK(do_project(c, L, g, vol, MGCT_F32, ax, sd, 0, 1, L.nviews, s, c.vt_dtype));
    HIPCHK(launch_residual(b, b_dtype, ax, r, sd, L.rays(), part, kRedBlocks, s));
    HIPCHK(launch_finish_sum(part, kRedBlocks, norm2_out ? norm2_out : nrm, s));
    MGCHK(do_backproject(c, L, g, r, sd, grad, MGCT_F32, 0, 1, L.nviews, s));
    MGCHK(do_precondition(c, L, g, grad, grad, f, s));
    if (update_out)
        HIPCHK(launch_scale(grad, update_out, (float)alpha, L.vox(), s));
    else
        HIPCHK(launch_axpy(vol, grad, alpha, L.vox(), s));
    return MGCT_OK;
}

// ||b - A vol||^2 over the judge's views (every L.judge_step-th view, in the
// staged projector's order; L.d_order_judge must exist)
int do_residual_norm2_judge(Ctx &c, Level &L, int g, const float *vol, const float *b, double *norm2_out,
                            hipStream_t s) {
    const size_t nblk = project_lds_blocks_judge(L);
    WS(pp, double, "judge_partials", nblk * 8, false);
    WS(pp2, double, "proj_partials2", 256 * 8, false);
    void *vt;
    MGCHK(plain_copy(c, L, g, vol, MGCT_F32, MGCT_F32, &vt, s));
    KernelTimer t(c, MGCT_OP_PROJECT, g, s);
    HIPCHK(launch_project_lds_mode(vt, MGCT_F32, 3, nullptr, MGCT_F32, b, MGCT_F32, pp, L, s, L.d_order_judge,
                                   L.n_t_judge));
    HIPCHK(launch_finish_sum_wide(pp, (int)nblk, pp2, norm2_out, s));
    return MGCT_OK;
}

int do_residual_norm2(Ctx &c, Level &L, int g, const float *vol, const float *b, double *norm2_out, hipStream_t s) {
    if (L.separable) {
        const bool lds = project_lds_ok(L, L.nviews, c.proj_variant);
        const size_t nblk = lds ? project_lds_blocks(L) : project_sep_blocks(L, L.nviews, MGCT_F32);
        WS(pp, double, "proj_partials", nblk * 8, false);
        WS(pp2, double, "proj_partials2", 256 * 8, false);
        if (lds) {
            void *vt;
            MGCHK(plain_copy(c, L, g, vol, MGCT_F32, MGCT_F32, &vt, s));
            KernelTimer t(c, MGCT_OP_PROJECT, g, s);
            HIPCHK(launch_project_lds_mode(vt, MGCT_F32, 3, nullptr, MGCT_F32, b, MGCT_F32, pp, L, s));
        } else {
            void *vtx, *vty;
            MGCHK(pair_copies(c, L, g, vol, MGCT_F32, MGCT_F32, &vtx, &vty, s));
            KernelTimer t(c, MGCT_OP_PROJECT, g, s);
            HIPCHK(launch_project_sep_mode(vtx, vty, MGCT_F32, 3, nullptr, nullptr, MGCT_F32, b, MGCT_F32, nullptr,
                                           pp, L, 0, 1, L.nviews, s));
        }
        HIPCHK(launch_finish_sum_wide(pp, (int)nblk, pp2, norm2_out, s));
        return MGCT_OK;
    }
    WS(ax, float, lvl("lw_ax", g), L.rays() * 4, false);
    WS(r, float, lvl("lw_r", g), L.rays() * 4, false);
    WS(part, double, "red_partials", kRedBlocks * 8, false);
    MGCHK(do_project(c, L, g, vol, MGCT_F32, ax, MGCT_F32, 0, 1, L.nviews, s));
    HIPCHK(launch_residual(b, MGCT_F32, ax, r, MGCT_F32, L.rays(), part, kRedBlocks, s));
    HIPCHK(launch_finish_sum(part, kRedBlocks, norm2_out, s));
    return MGCT_OK;
}

int do_osemtr(Ctx &c, Level &L, int g, float *vol, const float *b, int M, int passes, hipStream_t s) {
    const size_t n = L.vox(), per = (size_t)L.nu * L.nv;
    const int maxsub = (L.nviews + M - 1) / M;
    const int nsteps = passes * std::min(M, L.nviews);
    WS(ones, float, lvl("emtr_ones", g), n * 4, false);
    WS(pi, float, lvl("emtr_pi", g), L.rays() * 4, false);
    WS(l, float, lvl("emtr_l", g), maxsub * per * 4, false);
    WS(pt1, float, lvl("emtr_pt1", g), maxsub * per * 4, false);
    WS(num, float, lvl("emtr_num", g), n * 4, false);
    WS(den, float, lvl("emtr_den", g), n * 4, false);
    WS(mx, unsigned, "emtr_max", (size_t)nsteps * 4, false);
    WS(pt0, float, lvl("pt", g), (size_t)L.nviews * per * 4, false);
    // support projection A 1 (support = the whole grid); depends only on the
    // geometry and the storage precision, so it is kept until either changes
    if (!c.pi_valid[g]) {
        HIPCHK(launch_fill(ones, n, 1.f, s));
        MGCHK(do_project(c, L, g, ones, MGCT_F32, pi, MGCT_F32, 0, 1, L.nviews, s));
        c.pi_valid[g] = true;
    }
    // one max slot per subset step, cleared once (0.0f has all-zero bits)
    HIPCHK(launch_fill(reinterpret_cast<float *>(mx), nsteps, 0.f, s));
    if (L.separable) {
        // fused: the projector writes the subset's transposed, scaled EMTR
        // terms; the update refreshes the projector's pair copies in place
        void *vtx, *vty;
        MGCHK(pair_copies(c, L, g, vol, MGCT_F32, MGCT_F32, &vtx, &vty, s));
        int step = 0;
        for (int p = 0; p < passes; ++p) {
            for (int m = 0; m < M && m < L.nviews; ++m, ++step) {
                const int nsub = (L.nviews - m + M - 1) / M;
                {
                    KernelTimer t(c, MGCT_OP_PROJECT, g, s);
                    HIPCHK(launch_project_sep_mode(vtx, vty, MGCT_F32, 2, pt0, pt1, MGCT_F32, b, MGCT_F32, pi,
                                                   nullptr, L, m, M, nsub, s));
                }
                const size_t sb = backproject_scratch_bytes(L, nsub, 2);
                float *scratch = nullptr;
                if (sb) {
                    scratch = static_cast<float *>(workspace(c, lvl("bp_scratch2", g), sb, false));
                    if (!scratch) return MGCT_ERR_OOM;
                }
                int nchunks = 1;
                HIPCHK(launch_backproject2(pt0, pt1, num, den, scratch, L, m, M, nsub, s, &nchunks));
                const float *pn = nchunks > 1 ? scratch : nullptr;
                const float *pd = nchunks > 1 ? scratch + (size_t)nchunks * n : nullptr;
                HIPCHK(launch_emtr_reduce(pn, pd, num, den, n, nchunks, mx + step, s));
                HIPCHK(launch_emtr_update_pairs(vol, num, den, mx + step, vtx, vty, MGCT_F32, L, s));
            }
        }
        return MGCT_OK;
    }
    int step = 0;
    for (int p = 0; p < passes; ++p) {
        for (int m = 0; m < M && m < L.nviews; ++m, ++step) {
            const int nsub = (L.nviews - m + M - 1) / M;
            MGCHK(do_project(c, L, g, vol, MGCT_F32, l, MGCT_F32, m, M, nsub, s));
            HIPCHK(launch_emtr_terms_t(l, b, pi, pt0, pt1, L, m, M, nsub, s));
            int nchunks = 1;
            float *scratch = nullptr;
            if (L.separable) {
                const size_t sb = backproject_scratch_bytes(L, nsub, 2);
                if (sb) {
                    scratch = static_cast<float *>(workspace(c, lvl("bp_scratch2", g), sb, false));
                    if (!scratch) return MGCT_ERR_OOM;
                }
                HIPCHK(launch_backproject2(pt0, pt1, num, den, scratch, L, m, M, nsub, s, &nchunks));
            } else {
                const size_t sb = backproject_gen_scratch_bytes(L, nsub);
                if (sb) {
                    scratch = static_cast<float *>(workspace(c, lvl("bp_scratch", g), sb, false));
                    if (!scratch) return MGCT_ERR_OOM;
                }
                HIPCHK(launch_backproject_gen(pt0, MGCT_F32, num, scratch, L, m, M, nsub, s));
                HIPCHK(launch_backproject_gen(pt1, MGCT_F32, den, scratch, L, m, M, nsub, s));
            }
            const float *pn = nchunks > 1 ? scratch : nullptr;
            const float *pd = nchunks > 1 ? scratch + (size_t)nchunks * n : nullptr;
            HIPCHK(launch_emtr_reduce(pn, pd, num, den, n, nchunks, mx + step, s));
            HIPCHK(launch_emtr_update(vol, num, den, n, mx + step, s));
        }
    }
    return MGCT_OK;
}

// Key of a filter for the step-size cache.  A TRANSFER filter is keyed by the
// contents of grid g's array (an order-independent 64-bit hash computed on the
// device), not by its address: a new H(k) at the same address, or one
// rewritten in place, must not reuse an old step size.
int filter_key(Ctx &c, const mgct_filter *f, int g, const Level &L, hipStream_t s, std::string *out) {
    std::ostringstream o;
    if (!f || f->kind == MGCT_FILTER_IDENTITY) {
        *out = "id";
        return MGCT_OK;
    }
    o << f->kind << ":";
    if (f->kind == MGCT_FILTER_STENCIL27) {
        for (int i = 0; i < 27; ++i) o << f->taps[i] << ",";
    } else if (f->kind == MGCT_FILTER_TRANSFER) {
        constexpr int kHashBlocks = 256;
        WS(part, unsigned long long, "hash_partials", kHashBlocks * 8, false);
        WS(hd, unsigned long long, "hash_out", 8, false);
        HIPCHK(launch_hash_words(f->transfer[g], L.vox(), part, kHashBlocks, hd, s));
        unsigned long long h = 0;
        HIPCHK(hipMemcpyAsync(&h, hd, 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        o << L.vox() << "," << h;
    } else {
        o << f->n_table << "," << f->rho_max << ",";
        uint64_t hsh = 1469598103934665603ull;
        const unsigned char *p = (const unsigned char *)f->radial_table;
        for (size_t i = 0; i < (size_t)f->n_table * 4; ++i) hsh = (hsh ^ p[i]) * 1099511628211ull;
        o << hsh;
    }
    *out = o.str();
    return MGCT_OK;
}

// Divergence rule shared by the Landweber step and the multigrid solve.
bool diverged(double prev, double cur, double ratio) {
    if (!isfinite(cur)) return true;
    return ratio > 0.0 && prev > 0.0 && cur > ratio * prev;
}

int do_estimate(Ctx &c, Level &L, int g, const mgct_filter *f, int iters, uint64_t seed, double *alpha,
                hipStream_t s) {
    MGCHK(check_filter(f, L, g));
    const size_t n = L.vox();
    WS(x, float, lvl("pw_x", g), n * 4, false);
    WS(y, float, lvl("pw_y", g), n * 4, false);
    WS(p, float, lvl("pw_p", g), L.rays() * 4, false);
    WS(part, double, "red_partials", kRedBlocks * 8, false);
    WS(d, double, "pw_scalars", 16, false);
    HIPCHK(launch_splitmix_uniform(x, n, seed, s));
    HIPCHK(launch_sumsq(x, n, part, kRedBlocks, s));
    HIPCHK(launch_finish_sum(part, kRedBlocks, d, s));
    HIPCHK(launch_scale_by_inv_sqrt(x, n, d, nullptr, s));
    for (int it = 0; it < iters; ++it) {
        MGCHK(do_project(c, L, g, x, MGCT_F32, p, MGCT_F32, 0, 1, L.nviews, s));
        MGCHK(do_backproject(c, L, g, p, MGCT_F32, y, MGCT_F32, 0, 1, L.nviews, s));
        MGCHK(do_precondition(c, L, g, y, y, f, s));
        HIPCHK(launch_sumsq(y, n, part, kRedBlocks, s));
        HIPCHK(launch_finish_sum(part, kRedBlocks, d, s));
        HIPCHK(launch_scale_by_inv_sqrt(y, n, d, d + 1, s));
        float *t = x;
        x = y;
        y = t;
    }
    double lam = 0.0;
    HIPCHK(hipMemcpyAsync(&lam, d + 1, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (iters <= 0 || !(lam > 0.0) || !isfinite(lam)) return MGCT_ERR_DIVERGED;
    *alpha = 1.0 / lam;
    return MGCT_OK;
}

int cnn_buffers(Ctx &c, int nx, int ny, int nz, bool train, CnnBuffers &B) {
    auto get = [&](const char *name, size_t bytes, bool zero = false) { return workspace(c, name, bytes, zero); };
    const long n = (long)nx * ny * nz;
    B.up = (float *)get("cnn_up", (size_t)(nx + 2) * (ny + 2) * (nz + 2) * 4);
    B.h1 = (uint16_t *)get("cnn_h1", n * 16 * 2);
    B.h2 = (uint16_t *)get("cnn_h2", n * 32 * 2);
    B.h3 = (uint16_t *)get("cnn_h3", n * 32 * 2);
    if (!B.up || !B.h1 || !B.h2 || !B.h3) return MGCT_ERR_OOM;
    if (!train) return MGCT_OK;
    B.z1 = (float *)get("cnn_z1", n * 16 * 4);
    B.z2 = (float *)get("cnn_z2", n * 32 * 4);
    B.z3 = (float *)get("cnn_z3", n * 32 * 4);
    B.dout = (float *)get("cnn_dout", n * 4);
    B.dz3 = (uint16_t *)get("cnn_dz3", n * 32 * 2);
    B.dz2 = (uint16_t *)get("cnn_dz2", n * 32 * 2);
    B.dz1 = (uint16_t *)get("cnn_dz1", n * 16 * 2);
    B.gT = (uint16_t *)get("cnn_gT", n * 32 * 2);
    if (!B.z1 || !B.z2 || !B.z3 || !B.dout || !B.dz3 || !B.dz2 || !B.dz1 || !B.gT) return MGCT_ERR_OOM;
    return MGCT_OK;
}

// padded channels-first copy (its zero border must survive: allocated zeroed
// once per volume shape) and the partial-sum scratch
int cnn_train_scratch(Ctx &c, int nx, int ny, int nz, CnnBuffers &B) {
    const size_t padded = (size_t)(nx + 2) * (ny + 2) * (nz + 2) * 32 * 2;
    std::string key = "cnn_xT_" + std::to_string(nx) + "x" + std::to_string(ny) + "x" + std::to_string(nz);
    B.xT = (uint16_t *)workspace(c, key, padded, true);
    const long n = (long)nx * ny * nz;
    const long rows = (long)ny * nz, nch = (rows + 15) / 16;
    const long vchunk = std::max(512L, (n + 4095) / 4096), nvb = (n + vchunk - 1) / vchunk;  // as cnn_backward
    const long wrb = (long)(nx / 32) * ((rows + 3) / 4);  // VALU weight-gradient blocks (4 rows each)
    const size_t part = std::max({(size_t)nch * 27 * 1024, (size_t)nvb * 32, (size_t)wrb * 865}) * 4;
    B.partial = (float *)workspace(c, "cnn_partial", part);
    if (!B.xT || !B.partial) return MGCT_ERR_OOM;
    return MGCT_OK;
}

int cnn_check(Ctx &c, int nx, int ny, int nz) {
    if (!c.cnn.ready) return MGCT_ERR_INVALID_ARG;
    if (nx < 32 || ny < 1 || nz < 1 || nx % 32) return MGCT_ERR_INVALID_ARG;
    return MGCT_OK;
}

}  // namespace

// ======================================================================
extern "C" {

int mgct_learned_stats(void *ctx, int *accepted, int *rejected) {
    if (!ctx) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    unsigned *cnt = static_cast<unsigned *>(workspace(c, "learned_counters", 8, true));
    if (!cnt) return MGCT_ERR_OOM;
    unsigned h[2] = {0, 0};
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(h, cnt, 8, hipMemcpyDeviceToHost));
    HIPCHK(hipMemset(cnt, 0, 8));
    if (accepted) *accepted = (int)h[0];
    if (rejected) *rejected = (int)h[1];
    return MGCT_OK;
}

int mgct_learned_judge(void *ctx, double *r0, double *r1, int *view_step) {
    if (!ctx || !r0 || !r1) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    auto it = c.ws.find("mg_judge");
    if (it == c.ws.end() || c.judge_step_used == 0) return MGCT_ERR_INVALID_ARG;
    double h[2];
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(h, it->second.first, 16, hipMemcpyDeviceToHost));
    *r0 = h[0];
    *r1 = h[1];
    if (view_step) *view_step = c.judge_step_used;
    return MGCT_OK;
}

static int upload_shapes(Ctx &c, const double *ell, int K, const double *box, int J, double **de, double **db) {
    double *e = static_cast<double *>(workspace(c, "synth_ell", (size_t)(K > 0 ? K : 1) * 16 * 8));
    double *b = static_cast<double *>(workspace(c, "synth_box", (size_t)(J > 0 ? J : 1) * 7 * 8));
    if (!e || !b) return MGCT_ERR_OOM;
    if (K > 0) HIPCHK(hipMemcpy(e, ell, (size_t)K * 16 * 8, hipMemcpyHostToDevice));
    if (J > 0) HIPCHK(hipMemcpy(b, box, (size_t)J * 7 * 8, hipMemcpyHostToDevice));
    *de = e;
    *db = b;
    return MGCT_OK;
}

int mgct_synth_line_integrals(void *ctx, const double *ell, int K, const double *box, int J, float *out,
                              hipStream_t s) {
    if (!ctx || !out || K < 0 || J < 0 || (K && !ell) || (J && !box)) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    if (!c.has_geom) return MGCT_ERR_NO_GEOMETRY;
    double *de, *db;
    HIPCHK(hipStreamSynchronize(s));
    MGCHK(upload_shapes(c, ell, K, box, J, &de, &db));
    double *dv = static_cast<double *>(workspace(c, "synth_views", c.views.size() * 8));
    if (!dv) return MGCT_ERR_OOM;
    HIPCHK(hipMemcpy(dv, c.views.data(), c.views.size() * 8, hipMemcpyHostToDevice));
    HIPCHK(launch_synth_line_integrals(dv, c.nviews, c.nu, c.nv, de, K, db, J, out, s));
    return MGCT_OK;
}

int mgct_synth_voxelize(void *ctx, const double *ell, int K, const double *box, int J, int ss, float *vol,
                        hipStream_t s) {
    if (!ctx || !vol || K < 0 || J < 0 || ss < 1 || ss > 16 || (K && !ell) || (J && !box)) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    if (!c.has_geom) return MGCT_ERR_NO_GEOMETRY;
    double *de, *db;
    HIPCHK(hipStreamSynchronize(s));
    MGCHK(upload_shapes(c, ell, K, box, J, &de, &db));
    HIPCHK(launch_synth_voxelize(c.nx, c.ny, c.nz, c.h, c.origin, de, K, db, J, ss, vol, s));
    return MGCT_OK;
}

int mgct_cnn_set_weights(void *ctx, const float *w, int n) {
    if (!ctx || !w || n != kCnnParams) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    CnnState &S = c.cnn;
    if (!S.master) {
        void *p = nullptr;
        const size_t fb = kCnnParams * 4;
        if (hipMalloc(&p, 4 * fb + 2 * (size_t)27 * 32 * 16 + 3 * 2 * (size_t)27 * 32 * 32 + 2 * 6144 + 2 * 1536) !=
            hipSuccess)
            return MGCT_ERR_OOM;
        char *q = (char *)p;
        S.master = (float *)q; q += fb;
        S.adam_m = (float *)q; q += fb;
        S.adam_v = (float *)q; q += fb;
        S.grads = (float *)q; q += fb;
        S.p2f = (uint16_t *)q; q += 2 * 27 * 32 * 16;
        S.p3f = (uint16_t *)q; q += 2 * 27 * 32 * 32;
        S.p3d = (uint16_t *)q; q += 2 * 27 * 32 * 32;
        S.p2d = (uint16_t *)q; q += 2 * 27 * 32 * 32;
        S.p4 = (uint16_t *)q; q += 2 * 6144;
        S.p1 = (uint16_t *)q;
    }
    HIPCHK(hipMemcpy(S.master, w, kCnnParams * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemset(S.adam_m, 0, kCnnParams * 4));
    HIPCHK(hipMemset(S.adam_v, 0, kCnnParams * 4));
    S.adam_t = 0;
    HIPCHK(cnn_pack(S, 0));
    HIPCHK(hipDeviceSynchronize());
    S.ready = true;
    return MGCT_OK;
}

int mgct_cnn_get_weights(void *ctx, float *w, int n) {
    if (!ctx || !w || n != kCnnParams) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    if (!c.cnn.ready) return MGCT_ERR_INVALID_ARG;
    HIPCHK(hipSetDevice(c.device));
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(w, c.cnn.master, kCnnParams * 4, hipMemcpyDeviceToHost));
    return MGCT_OK;
}

int mgct_cnn_forward(void *ctx, int nx, int ny, int nz, const float *u, float *out, hipStream_t s) {
    if (!ctx || !u || !out) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    MGCHK(cnn_check(c, nx, ny, nz));
    CnnBuffers B;
    MGCHK(cnn_buffers(c, nx, ny, nz, false, B));
    HIPCHK(cnn_forward(c.cnn, B, u, out, nx, ny, nz, false, s));
    return MGCT_OK;
}

static int cnn_fwd_bwd(Ctx &c, int nx, int ny, int nz, const float *u, const float *target, double *loss,
                       hipStream_t s) {
    const long n = (long)nx * ny * nz;
    CnnBuffers B;
    MGCHK(cnn_buffers(c, nx, ny, nz, true, B));
    MGCHK(cnn_train_scratch(c, nx, ny, nz, B));
    WS(out, float, "cnn_out", n * 4, false);
    WS(part, double, "red_partials", kRedBlocks * 8, false);
    WS(lsum, double, "cnn_loss", 8, false);
    HIPCHK(cnn_forward(c.cnn, B, u, out, nx, ny, nz, true, s));
    HIPCHK(cnn_backward(c.cnn, B, u, out, target, c.cnn.grads, part, kRedBlocks, nx, ny, nz, s));
    HIPCHK(launch_finish_sum(part, kRedBlocks, lsum, s));
    if (loss) {
        double v = 0.0;
        HIPCHK(hipMemcpyAsync(&v, lsum, 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        *loss = v / (double)n;
    }
    return MGCT_OK;
}

int mgct_cnn_gradients(void *ctx, int nx, int ny, int nz, const float *u, const float *target, float *grads,
                       double *loss, hipStream_t s) {
    if (!ctx || !u || !target || !grads) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    MGCHK(cnn_check(c, nx, ny, nz));
    MGCHK(cnn_fwd_bwd(c, nx, ny, nz, u, target, loss, s));
    HIPCHK(hipMemcpyAsync(grads, c.cnn.grads, kCnnParams * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return MGCT_OK;
}

int mgct_cnn_backward(void *ctx, int nx, int ny, int nz, const float *u, const float *dout, float *grads,
                      hipStream_t s) {
    if (!ctx || !u || !dout || !grads) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    MGCHK(cnn_check(c, nx, ny, nz));
    const long n = (long)nx * ny * nz;
    CnnBuffers B;
    MGCHK(cnn_buffers(c, nx, ny, nz, true, B));
    MGCHK(cnn_train_scratch(c, nx, ny, nz, B));
    WS(out, float, "cnn_out", n * 4, false);
    // the activations of u (recomputed), then the backward pass from dout
    HIPCHK(cnn_forward(c.cnn, B, u, out, nx, ny, nz, true, s));
    HIPCHK(hipMemcpyAsync(B.dout, dout, n * 4, hipMemcpyDeviceToDevice, s));
    HIPCHK(cnn_backward(c.cnn, B, u, out, nullptr, c.cnn.grads, nullptr, 0, nx, ny, nz, s));
    HIPCHK(hipMemcpyAsync(grads, c.cnn.grads, kCnnParams * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return MGCT_OK;
}

int mgct_adam_step(void *ctx, const float *grads, int n, double lr, hipStream_t s) {
    if (!ctx || !grads || n != kCnnParams || !(lr > 0.0)) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    if (!c.cnn.ready) return MGCT_ERR_INVALID_ARG;
    HIPCHK(hipMemcpyAsync(c.cnn.grads, grads, kCnnParams * 4, hipMemcpyHostToDevice, s));
    HIPCHK(cnn_adam(c.cnn, c.cnn.grads, (float)lr, s));
    HIPCHK(hipStreamSynchronize(s));
    return MGCT_OK;
}

int mgct_cnn_train_step(void *ctx, int nx, int ny, int nz, const float *u, const float *target, double lr,
                        double *loss, hipStream_t s) {
    if (!ctx || !u || !target || !(lr > 0.0)) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    MGCHK(cnn_check(c, nx, ny, nz));
    MGCHK(cnn_fwd_bwd(c, nx, ny, nz, u, target, loss, s));
    HIPCHK(cnn_adam(c.cnn, c.cnn.grads, (float)lr, s));
    return MGCT_OK;
}


const char *mgct_status_string(int st) {
    switch (st) {
        case MGCT_OK: return "ok";
        case MGCT_ERR_INVALID_ARG: return "invalid argument";
        case MGCT_ERR_UNSUPPORTED_GEOMETRY: return "unsupported geometry (z-major ray or source inside the volume)";
        case MGCT_ERR_SIZE_NOT_DIVISIBLE: return "size not divisible by 2^level";
        case MGCT_ERR_OOM: return "device allocation failed";
        case MGCT_ERR_HIP: return "HIP runtime error";
        case MGCT_ERR_DIVERGED: return "iteration diverged (residual grew or is not finite, or no positive spectrum estimate)";
        case MGCT_ERR_TOO_LARGE: return "grid exceeds the fixed scratch of the allocation-free entry point";
        case MGCT_ERR_NOT_IMPLEMENTED: return "not implemented for these arguments";
        case MGCT_ERR_NO_GEOMETRY: return "no geometry set";
        default: return "unknown status";
    }
}

int mgct_filter_eq5(mgct_filter *f) {
    if (!f) return MGCT_ERR_INVALID_ARG;
    static const float outer[9] = {-1, -1, -1, -1, 0, -1, -1, -1, -1};
    static const float middle[9] = {-8, -4, -8, -4, 64, -4, -8, -4, -8};
    memset(f, 0, sizeof(*f));
    f->kind = MGCT_FILTER_STENCIL27;
    for (int i = 0; i < 9; ++i) {
        f->taps[i] = outer[i] / 64.f;
        f->taps[9 + i] = middle[i] / 64.f;
        f->taps[18 + i] = outer[i] / 64.f;
    }
    return MGCT_OK;
}

int mgct_create(int device, void **ctx_out) {
    if (!ctx_out) return MGCT_ERR_INVALID_ARG;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return MGCT_ERR_INVALID_ARG;
    HIPCHK(hipSetDevice(device));
    MGCHK(static_scratch_setup(device));
    Ctx *c = new Ctx();
    c->device = device;
    *ctx_out = c;
    return MGCT_OK;
}

static void release_events(Ctx &c) {
    for (auto &r : c.timed) {
        c.event_pool.push_back(r.start);
        c.event_pool.push_back(r.stop);
    }
    c.timed.clear();
}

int mgct_kernel_timing(void *ctx, int enable) {
    if (!ctx) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    if (enable) {
        HIPCHK(hipDeviceSynchronize());
        release_events(c);
    }
    c.timing = enable != 0;
    return MGCT_OK;
}

int mgct_kernel_timing_select(void *ctx, unsigned op_mask, unsigned level_mask) {
    if (!ctx) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    c.timing_ops = op_mask;
    c.timing_levels = level_mask;
    return MGCT_OK;
}

int mgct_kernel_time(void *ctx, int op, int level, double *total_ms, int *launches) {
    if (!ctx || !total_ms || op < 0 || op >= MGCT_OP_COUNT) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    double tot = 0.0;
    int n = 0;
    for (auto &r : c.timed) {
        if (r.op != op || (level >= 0 && r.level != level)) continue;
        HIPCHK(hipEventSynchronize(r.stop));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, r.start, r.stop));
        tot += ms;
        ++n;
    }
    *total_ms = tot;
    if (launches) *launches = n;
    return MGCT_OK;
}

int mgct_destroy(void *ctx) {
    if (!ctx) return MGCT_ERR_INVALID_ARG;
    Ctx *c = as_ctx(ctx);
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    release_events(*c);
    for (auto e : c->event_pool) (void)hipEventDestroy(e);
    if (c->cnn.master) (void)hipFree(c->cnn.master);
    for (auto &kv : c->ws) (void)hipFree(kv.second.first);
    for (auto &L : c->levels) free_level(L);
    delete c;
    return MGCT_OK;
}

int mgct_set_geometry(void *ctx, int nx, int ny, int nz, double voxel, const double origin[3], int nu, int nv,
                      int n_views, const double *views) {
    if (!ctx) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    MGCHK(check_geometry(nx, ny, nz, voxel, origin, nu, nv, n_views, views));
    HIPCHK(hipDeviceSynchronize());
    for (auto &L : c.levels) {
        free_level(L);
        L = Level();
    }
    // The projector's padded volume copies rely on zero borders that are
    // written only when a workspace is first allocated; another grid shape
    // would place earlier interior voxels in the new borders.  A change of
    // shape therefore releases every workspace (the same shape keeps them).
    if (!c.has_geom || c.nx != nx || c.ny != ny || c.nz != nz) {
        for (auto &w : c.ws) (void)hipFree(w.second.first);
        c.ws.clear();
    }
    for (auto &ch : c.lw_chain) ch = Ctx::LwChain();
    c.alpha_cache.clear();
    for (bool &v : c.pi_valid) v = false;
    c.nx = nx; c.ny = ny; c.nz = nz; c.nu = nu; c.nv = nv; c.nviews = n_views;
    c.h = voxel;
    for (int k = 0; k < 3; ++k) c.origin[k] = origin[k];
    c.views.assign(views, views + (size_t)n_views * 12);
    c.has_geom = true;
    Level *L = nullptr;
    int r = get_level(c, 0, &L);
    if (r != MGCT_OK) c.has_geom = false;
    return r;
}

int mgct_set_precision(void *ctx, int volume_copy_dtype, int stack_dtype) {
    if (!ctx || !vol_dtype_ok(volume_copy_dtype) || !stack_dtype_ok(stack_dtype)) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    c.vt_dtype = volume_copy_dtype;
    c.stack_dtype = stack_dtype;
    for (bool &v : c.pi_valid) v = false;
    return MGCT_OK;
}

int mgct_project(void *ctx, int level, const void *vol, int vol_dtype, void *proj, int proj_dtype, hipStream_t s) {
    if (!ctx || !vol || !proj || !vol_dtype_ok(vol_dtype) || !stack_dtype_ok(proj_dtype)) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    Level *L;
    MGCHK(get_level(c, level, &L));
    return do_project(c, *L, level, vol, vol_dtype, proj, proj_dtype, 0, 1, L->nviews, s);
}

int mgct_backproject(void *ctx, int level, const void *proj, int proj_dtype, void *vol, int vol_dtype,
                     hipStream_t s) {
    if (!ctx || !vol || !proj || !vol_dtype_ok(vol_dtype) || !stack_dtype_ok(proj_dtype)) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    Level *L;
    MGCHK(get_level(c, level, &L));
    return do_backproject(c, *L, level, proj, proj_dtype, vol, vol_dtype, 0, 1, L->nviews, s);
}

int mgct_precondition(void *ctx, int level, const float *in, float *out, const mgct_filter *f, hipStream_t s) {
    if (!ctx || !in || !out) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    Level *L;
    MGCHK(get_level(c, level, &L));
    return do_precondition(c, *L, level, in, out, f, s);
}

int mgct_estimate_step(void *ctx, int level, const mgct_filter *f, int iters, uint64_t seed, double *alpha,
                       hipStream_t s) {
    if (!ctx || !alpha || iters < 1) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    Level *L;
    MGCHK(get_level(c, level, &L));
    return do_estimate(c, *L, level, f, iters, seed, alpha, s);
}

int mgct_landweber_step(void *ctx, int level, float *vol, const void *b, int b_dtype, double alpha,
                        const mgct_filter *f, double *resid_norm, hipStream_t s) {
    if (!ctx || !vol || !b || !stack_dtype_ok(b_dtype) || !isfinite(alpha)) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    Level *L;
    MGCHK(get_level(c, level, &L));
    MGCHK(check_filter(f, *L, level));
    WS(d, double, "lw_norm2", 8, false);
    MGCHK(do_landweber(c, *L, level, vol, b, b_dtype, alpha, f, d, s));
    if (resid_norm) {
        double v = 0.0;
        HIPCHK(hipMemcpyAsync(&v, d, 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        *resid_norm = sqrt(v);
        // eq. 2 / eq. 4 with p positive semi-definite: for alpha <= 2/lambda_max
        // the residual cannot grow from one step to the next
        std::string fk;
        MGCHK(filter_key(c, f, level, *L, s, &fk));
        Ctx::LwChain &ch = c.lw_chain[level];
        const bool same = ch.valid && ch.b == b && ch.alpha == alpha && ch.filter == fk;
        const bool bad = diverged(same ? ch.prev : 0.0, *resid_norm, c.diverge_ratio);
        ch.valid = true;
        ch.b = b;
        ch.alpha = alpha;
        ch.filter = fk;
        ch.prev = *resid_norm;
        if (bad) return MGCT_ERR_DIVERGED;
    }
    return MGCT_OK;
}

int mgct_set_projector(void *ctx, int variant) {
    if (!ctx || variant < MGCT_PROJECTOR_AUTO || variant > MGCT_PROJECTOR_STAGED) return MGCT_ERR_INVALID_ARG;
    as_ctx(ctx)->proj_variant = variant;
    return MGCT_OK;
}

int mgct_set_divergence(void *ctx, double ratio) {
    if (!ctx || !(ratio == 0.0 || ratio >= 1.0) || !isfinite(ratio)) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    c.diverge_ratio = ratio;
    for (auto &ch : c.lw_chain) ch = Ctx::LwChain();
    return MGCT_OK;
}

int mgct_residual_diverged(double prev, double cur, double ratio) { return diverged(prev, cur, ratio) ? 1 : 0; }

int mgct_project_geom_grad(void *ctx, int level, const float *vol, const float *cot, double *dviews, hipStream_t s) {
    if (!ctx || !vol || !cot || !dviews) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    Level *Lp;
    MGCHK(get_level(c, level, &Lp));
    Level &L = *Lp;
    // the derivative kernel addresses its padded FP32 copy with 32-bit byte offsets
    if (L.padded_vox() * 4 > 0xFFFFFFF0ull) return MGCT_ERR_NOT_IMPLEMENTED;
    void *vt = workspace(c, lvl("vt32", level), L.padded_vox() * 4 + kCopyTail, true);
    if (!vt) return MGCT_ERR_OOM;
    WS(partial, double, lvl("gg_partial", level), geom_grad_partial_bytes(L), false);
    WS(dv, double, lvl("gg_dviews", level), (size_t)L.nviews * 12 * 8, false);
    HIPCHK(launch_transpose_volume(vol, MGCT_F32, vt, MGCT_F32, L, s));
    HIPCHK(launch_geom_grad(vt, MGCT_F32, cot, partial, dv, L, s));
    HIPCHK(hipMemcpyAsync(dviews, dv, (size_t)L.nviews * 12 * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return MGCT_OK;
}

int mgct_geometry_param_grad(int n_views, const double *views0, const double *dviews, double voxel, double dx,
                             double dz, double tilt_deg, double grad[3]) {
    if (n_views < 1 || !views0 || !dviews || !grad || !(voxel > 0.0)) return MGCT_ERR_INVALID_ARG;
    const double t = tilt_deg * M_PI / 180.0, ct = cos(t), st = sin(t), k = M_PI / 180.0;
    double g0 = 0.0, g1 = 0.0, g2 = 0.0;
    for (int v = 0; v < n_views; ++v) {
        const double *w = views0 + (size_t)v * 12, *d = dviews + (size_t)v * 12;
        double lu = sqrt(w[6] * w[6] + w[7] * w[7] + w[8] * w[8]);
        double lv = sqrt(w[9] * w[9] + w[10] * w[10] + w[11] * w[11]);
        double uh[3] = {w[6] / lu, w[7] / lu, w[8] / lu}, vh[3] = {w[9] / lv, w[10] / lv, w[11] / lv};
        for (int e = 0; e < 3; ++e) {
            g0 += d[e] * voxel * uh[e];                                 // source along the unit column direction
            g2 += d[6 + e] * k * lu * (-st * uh[e] + ct * vh[e]);       // column step rotates
            g2 += d[9 + e] * k * lv * (-ct * uh[e] - st * vh[e]);       // row step rotates
        }
        g1 += d[2] * voxel;                                             // source along z
    }
    grad[0] = g0;
    grad[1] = g1;
    grad[2] = g2;
    return MGCT_OK;
}

int mgct_psf_spectrum(void *ctx, int level, float *T, hipStream_t s) {
    if (!ctx || !T) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    Level *Lp;
    MGCHK(get_level(c, level, &Lp));
    Level &L = *Lp;
    if (!fft_size_ok(L.nx) || !fft_size_ok(L.ny) || !fft_size_ok(L.nz)) return MGCT_ERR_NOT_IMPLEMENTED;
    const size_t n = L.vox();
    WS(delta, float, lvl("psf_delta", level), n * 4, false);
    WS(proj, float, lvl("psf_proj", level), L.rays() * 4, false);
    WS(work, float2, "fft_work", n * sizeof(float2), false);
    float2 *tw;
    MGCHK(fft_twiddles(c, L, &tw));
    HIPCHK(launch_fill(delta, n, 0.f, s));
    const float one = 1.f;
    const size_t centre = ((size_t)(L.nz / 2) * L.ny + L.ny / 2) * L.nx + L.nx / 2;
    HIPCHK(hipMemcpyAsync(delta + centre, &one, 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));  // `one` lives on this stack frame
    MGCHK(do_project(c, L, level, delta, MGCT_F32, proj, MGCT_F32, 0, 1, L.nviews, s));
    MGCHK(do_backproject(c, L, level, proj, MGCT_F32, delta, MGCT_F32, 0, 1, L.nviews, s));
    HIPCHK(launch_radial_filter(delta, nullptr, work, L.nx, L.ny, L.nz, nullptr, 0, 1.f, tw, s, nullptr, true));
    HIPCHK(launch_spectrum_real(work, T, L.nx, L.ny, L.nz, s));
    return MGCT_OK;
}

int mgct_transfer_from_spectrum(void *ctx, int level, const float *T, double floor_rel, float *H, hipStream_t s) {
    if (!ctx || !T || !H || T == H || !(floor_rel > 0.0)) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    Level *L;
    MGCHK(get_level(c, level, &L));
    HIPCHK(launch_transfer_inverse(T, H, (long)L->vox(), floor_rel, s));
    return MGCT_OK;
}

int mgct_radial_profile(void *ctx, int level, const float *T, int n_table, double rho_max, double *profile,
                        int *counts, hipStream_t s) {
    if (!ctx || !T || !profile || n_table < 2 || !(rho_max > 0.0)) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    Level *L;
    MGCHK(get_level(c, level, &L));
    WS(sums, unsigned long long, "prof_sums", (size_t)n_table * 8, false);
    WS(cnt, unsigned, "prof_counts", (size_t)n_table * 4, false);
    HIPCHK(launch_fill(reinterpret_cast<float *>(sums), (size_t)n_table * 2, 0.f, s));
    HIPCHK(launch_fill(reinterpret_cast<float *>(cnt), (size_t)n_table, 0.f, s));
    const double scale = 16777216.0;  // 2^24
    HIPCHK(launch_radial_bin(T, L->nx, L->ny, L->nz, n_table, (float)rho_max, scale, sums, cnt, s));
    std::vector<unsigned long long> hs(n_table);
    std::vector<unsigned> hc(n_table);
    HIPCHK(hipMemcpyAsync(hs.data(), sums, (size_t)n_table * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hc.data(), cnt, (size_t)n_table * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int i = 0; i < n_table; ++i) {
        profile[i] = hc[i] ? (double)(long long)hs[i] / scale / (double)hc[i] : NAN;
        if (counts) counts[i] = (int)hc[i];
    }
    return MGCT_OK;
}

int mgct_restrict_volume(void *ctx, int level, const float *fine, float *coarse, hipStream_t s) {
    if (!ctx || !fine || !coarse) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    Level *L, *Lc;
    MGCHK(get_level(c, level, &L));
    MGCHK(get_level(c, level + 1, &Lc));
    HIPCHK(launch_restrict_volume(fine, coarse, L->nx, L->ny, L->nz, s));
    return MGCT_OK;
}

int mgct_restrict_stack(void *ctx, int level, const float *fine, float *coarse, hipStream_t s) {
    if (!ctx || !fine || !coarse) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    Level *L, *Lc;
    MGCHK(get_level(c, level, &L));
    MGCHK(get_level(c, level + 1, &Lc));
    HIPCHK(launch_restrict_stack(fine, coarse, L->nviews, L->nv, L->nu, s));
    return MGCT_OK;
}

int mgct_prolong_add(void *ctx, int level, const float *coarse_new, const float *coarse_old, float *fine,
                     hipStream_t s) {
    if (!ctx || !coarse_new || !coarse_old || !fine) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    Level *L, *Lc;
    MGCHK(get_level(c, level, &L));
    MGCHK(get_level(c, level + 1, &Lc));
    HIPCHK(launch_prolong_add(coarse_new, coarse_old, fine, L->nx, L->ny, L->nz, s));
    return MGCT_OK;
}

int mgct_soft_threshold(void *ctx, int level, float *vol, double lambda, hipStream_t s) {
    if (!ctx || !vol || !(lambda >= 0.0)) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    Level *L;
    MGCHK(get_level(c, level, &L));
    HIPCHK(launch_soft_threshold(vol, L->vox(), (float)lambda, s));
    return MGCT_OK;
}

int mgct_bilateral(void *ctx, int level, const float *in, float *out, double sigma_s, double sigma_r,
                   hipStream_t s) {
    if (!ctx || !in || !out || in == out || !(sigma_s > 0.0) || !(sigma_r > 0.0)) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    Level *L;
    MGCHK(get_level(c, level, &L));
    HIPCHK(launch_bilateral(in, out, L->nx, L->ny, L->nz, (float)sigma_s, (float)sigma_r, s));
    return MGCT_OK;
}

int mgct_osemtr(void *ctx, int level, float *vol, const float *b, int subsets, int passes, hipStream_t s) {
    if (!ctx || !vol || !b || subsets < 1 || passes < 0) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    Level *L;
    MGCHK(get_level(c, level, &L));
    return do_osemtr(c, *L, level, vol, b, subsets, passes, s);
}

int mgct_multigrid_solve(void *ctx, float *vol, const void *b, int b_dtype, const mgct_mg_params *p,
                         double *resid_hist, hipStream_t s) {
    if (!ctx || !vol || !b || !p || !stack_dtype_ok(b_dtype)) return MGCT_ERR_INVALID_ARG;
    if (p->levels < 1 || p->levels > 8 || p->n_outer < 0) return MGCT_ERR_INVALID_ARG;
    if (p->levels >= 2 && (p->coarse_subsets < 1 || p->coarse_passes < 0)) return MGCT_ERR_INVALID_ARG;
    if (p->lambda < 0.0 || (p->bilateral_on && !(p->sigma_s > 0.0 && p->sigma_r > 0.0))) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    const int NL = p->levels;
    std::vector<Level *> Ls(NL);
    for (int g = 0; g < NL; ++g) MGCHK(get_level(c, g, &Ls[g]));
    const int nland = NL == 1 ? 1 : NL - 1;  // grids with a Landweber step
    for (int g = 0; g < nland; ++g) MGCHK(check_filter(&p->filter, *Ls[g], g));
    if (p->learned && (!c.cnn.ready || Ls[0]->nx % 32)) return MGCT_ERR_INVALID_ARG;

    // step sizes
    std::vector<double> alpha(nland);
    for (int g = 0; g < nland; ++g) {
        if (p->alpha[g] > 0.0) {
            alpha[g] = p->alpha[g];
            continue;
        }
        std::string fk;
        MGCHK(filter_key(c, &p->filter, g, *Ls[g], s, &fk));
        std::string key = std::to_string(g) + "|" + fk + "|" + std::to_string(p->power_iters) + "|" +
                          std::to_string(p->power_seed);
        auto it = c.alpha_cache.find(key);
        if (it != c.alpha_cache.end()) {
            alpha[g] = it->second;
        } else {
            if (p->power_iters < 1) return MGCT_ERR_INVALID_ARG;
            MGCHK(do_estimate(c, *Ls[g], g, &p->filter, p->power_iters, p->power_seed, &alpha[g], s));
            c.alpha_cache[key] = alpha[g];
        }
    }

    // data pyramid (FP32)
    std::vector<const float *> data(NL);
    if (b_dtype == MGCT_F32) {
        data[0] = (const float *)b;
    } else {
        WS(b0, float, "mg_b0", Ls[0]->rays() * 4, false);
        HIPCHK(launch_convert_to_f32(b, b_dtype, b0, Ls[0]->rays(), s));
        data[0] = b0;
    }
    for (int g = 1; g < NL; ++g) {
        WS(bg, float, lvl("mg_b", g), Ls[g]->rays() * 4, false);
        HIPCHK(launch_restrict_stack(data[g - 1], bg, Ls[g - 1]->nviews, Ls[g - 1]->nv, Ls[g - 1]->nu, s));
        data[g] = bg;
    }
    std::vector<float *> mu(NL), c0(NL);
    mu[0] = vol;
    for (int g = 1; g < NL; ++g) {
        WS(m, float, lvl("mg_mu", g), Ls[g]->vox() * 4, false);
        WS(o, float, lvl("mg_c0", g), Ls[g]->vox() * 4, false);
        mu[g] = m;
        c0[g] = o;
    }
    const int nh = p->n_outer * NL;
    WS(dh, double, "mg_hist", (size_t)(nh > 0 ? nh : 1) * 8, false);

    const float lam = (float)p->lambda;
    std::function<int(int, int)> mg = [&](int g, int n) -> int {
        Level &L = *Ls[g];
        if (g + 1 < NL) {
            Level &Lc = *Ls[g + 1];
            HIPCHK(launch_restrict_volume(mu[g], c0[g + 1], L.nx, L.ny, L.nz, s));
            HIPCHK(launch_copy(c0[g + 1], mu[g + 1], Lc.vox(), s));
            if (g + 1 < NL - 1) {
                MGCHK(mg(g + 1, n));
            } else {
                if (resid_hist) MGCHK(do_residual_norm2(c, Lc, g + 1, mu[g + 1], data[g + 1], dh + n * NL + g + 1, s));
                MGCHK(do_osemtr(c, Lc, g + 1, mu[g + 1], data[g + 1], p->coarse_subsets, p->coarse_passes, s));
            }
            HIPCHK(launch_prolong_add(mu[g + 1], c0[g + 1], mu[g], L.nx, L.ny, L.nz, s));
        }
        if (g == 0 && (p->learned || p->capture_update || p->capture_iterate)) {
            // finest grid: filtered update u; optionally the network's
            // refinement, kept only if it lowers the residual
            WS(u, float, "mg_u", L.vox() * 4, false);
            double *r0 = dh + n * NL;
            MGCHK(do_landweber(c, L, 0, mu[0], data[0], MGCT_F32, alpha[0], &p->filter, r0, s, u));
            if (p->capture_update) HIPCHK(launch_copy(u, p->capture_update, L.vox(), s));
            if (p->capture_iterate) HIPCHK(launch_copy(mu[0], p->capture_iterate, L.vox(), s));
            if (p->learned) {
                // The judge keeps the network's refinement only if it lowers
                // ||b - A mu||^2 below its value before the update.  On scans
                // of 720 views or more it compares both over every
                // judge_step-th view (about 360): the value before the update
                // is then the sum of the Landweber projection's block
                // partials over those views, and the one after it one staged
                // projection of those views.  Otherwise over all views.
                WS(cu, float, "mg_cnn_out", L.vox() * 4, false);
                WS(try_mu, float, "mg_try", L.vox() * 4, false);
                WS(jr, double, "mg_judge", 16, false);  // the two squared norms compared
                WS(cnt, unsigned, "learned_counters", 8, true);
                const bool sub = L.judge_step > 1 && L.d_order_judge && project_lds_ok(L, L.nviews, c.proj_variant);
                if (sub) {
                    const size_t nblk = project_lds_blocks(L);
                    const int n_t = L.n_rt * L.nviews;
                    WS(pp, double, "proj_partials", nblk * 8, false);
                    WS(pp2, double, "proj_partials2", 256 * 8, false);
                    HIPCHK(launch_finish_sum_views(pp, L.d_order, (int)(nblk / n_t), n_t, L.n_rt, L.judge_step, pp2,
                                                   jr, s));
                } else {
                    HIPCHK(hipMemcpyAsync(jr, r0, 8, hipMemcpyDeviceToDevice, s));
                }
                CnnBuffers B;
                MGCHK(cnn_buffers(c, L.nx, L.ny, L.nz, false, B));
                HIPCHK(cnn_forward(c.cnn, B, u, cu, L.nx, L.ny, L.nz, false, s));
                HIPCHK(launch_add(mu[0], cu, try_mu, L.vox(), s));
                if (sub)
                    MGCHK(do_residual_norm2_judge(c, L, 0, try_mu, data[0], jr + 1, s));
                else
                    MGCHK(do_residual_norm2(c, L, 0, try_mu, data[0], jr + 1, s));
                HIPCHK(launch_select_update(mu[0], u, try_mu, L.vox(), jr, jr + 1, cnt, s));
                c.judge_step_used = sub ? L.judge_step : 1;
            } else {
                HIPCHK(launch_axpy(mu[0], u, 1.0, L.vox(), s));
            }
        } else {
            MGCHK(do_landweber(c, L, g, mu[g], data[g], MGCT_F32, alpha[g], &p->filter, dh + n * NL + g, s));
        }
        if (lam > 0.f) HIPCHK(launch_soft_threshold(mu[g], L.vox(), lam, s));
        if (p->bilateral_on) {
            WS(tmp, float, lvl("bf_tmp", g), L.vox() * 4, false);
            HIPCHK(launch_bilateral(mu[g], tmp, L.nx, L.ny, L.nz, (float)p->sigma_s, (float)p->sigma_r, s));
            HIPCHK(launch_copy(tmp, mu[g], L.vox(), s));
        }
        return MGCT_OK;
    };
    for (int n = 0; n < p->n_outer; ++n) MGCHK(mg(0, n));
    if (resid_hist && nh > 0) {
        std::vector<double> h(nh);
        HIPCHK(hipMemcpyAsync(h.data(), dh, nh * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int i = 0; i < nh; ++i) resid_hist[i] = sqrt(h[i]);
        // the fine grid's residual between outer iterations, and every
        // recorded residual's finiteness
        for (int i = 0; i < nh; ++i)
            if (!isfinite(resid_hist[i])) return MGCT_ERR_DIVERGED;
        for (int n = 1; n < p->n_outer; ++n)
            if (diverged(resid_hist[(n - 1) * NL], resid_hist[n * NL], c.diverge_ratio)) return MGCT_ERR_DIVERGED;
    }
    return MGCT_OK;
}

}  // extern "C"

// ======================================================================
// Allocation-free projection: the fixed scratch and its entry point.
//
// One array per GPU, in the code object's device memory, holds the
// projector's padded volume copies for mgct_project_noalloc.  Its device
// address is looked up once per device (with that device current) when a
// context is created there, and only that address is used from the host: the
// array's name in host code is a host-side stand-in, not a device address.
namespace {
constexpr size_t kStaticScratchBytes = 40ull << 20;  // 40 MiB: FP32 pair copies of grids up to 128^3
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};

void *static_scratch(int device) {
    if (device < 0 || device >= kMaxScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
}  // namespace

static int static_scratch_setup(int device) {
    if (device < 0 || device >= kMaxScratchDevices) return MGCT_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return MGCT_OK;
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return MGCT_ERR_HIP;
    g_scratch_ptr[device] = ptr;
    return MGCT_OK;
}

extern "C" {

int mgct_project_noalloc(void *ctx, int level, const void *vol, int vol_dtype, void *proj, int proj_dtype,
                         hipStream_t s) {
    if (!ctx || !vol || !proj || !vol_dtype_ok(vol_dtype) || !stack_dtype_ok(proj_dtype)) return MGCT_ERR_INVALID_ARG;
    Ctx &c = *as_ctx(ctx);
    HIPCHK(hipSetDevice(c.device));
    if (!c.has_geom) return MGCT_ERR_NO_GEOMETRY;
    if (level < 0 || level >= Ctx::kMaxLevels) return MGCT_ERR_INVALID_ARG;
    Level &L = c.levels[level];
    if (L.nx == 0) return MGCT_ERR_INVALID_ARG;  // the grid's tables are built by an earlier call
    char *base = static_cast<char *>(static_scratch(c.device));
    if (!base) return MGCT_ERR_HIP;
    // the projector's copy has the input's type, as in mgct_project
    const int vt = vol_dtype;
    const size_t es = vt == MGCT_F32 ? 4 : 2;
    if (L.separable) {
        const size_t one = align256(pair_copy_elems(L) * es);
        if (2 * one > kStaticScratchBytes) return MGCT_ERR_TOO_LARGE;
        // the copies' zero borders: the scratch keeps the previous call's contents
        HIPCHK(launch_fill(reinterpret_cast<float *>(base), 2 * one / 4, 0.f, s));
        HIPCHK(launch_transpose_pairs(vol, vol_dtype, base, base + one, vt, L, s));
        HIPCHK(launch_project_sep(base, base + one, vt, proj, proj_dtype, L, 0, 1, L.nviews, s));
        return MGCT_OK;
    }
    const size_t one = align256(L.padded_vox() * es);
    if (one > kStaticScratchBytes) return MGCT_ERR_TOO_LARGE;
    HIPCHK(launch_fill(reinterpret_cast<float *>(base), one / 4, 0.f, s));
    HIPCHK(launch_transpose_volume(vol, vol_dtype, base, vt, L, s));
    HIPCHK(launch_project(base, vt, proj, proj_dtype, L, 0, 1, L.nviews, s));
    return MGCT_OK;
}

}  // extern "C"
