// Host-side geometry tables for each grid level, in FP64.
//
// The major axis of every ray (the axis whose voxel-centre planes carry the
// ray's samples in Joseph's method) is decided here, once, in double
// precision, from the pixel centre d + (a-(nu-1)/2) u + (b-(nv-1)/2) v and
// the source s with ties going to x, then y, then z.  Both the projector and
// the back-projector read this table, so they always agree on the decision.
// Compiled with -ffp-contract=off so that the decision is the plain IEEE
// evaluation of that expression.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "mgct_internal.h"

namespace mgct {

static int major_axis_phys(const double D[3]) {
    double ax = fabs(D[0]), ay = fabs(D[1]), az = fabs(D[2]);
    if (ax >= ay && ax >= az) return 0;
    if (ay >= az) return 1;
    return 2;
}

static void ray_dir(const double *view, int nu, int nv, int a, int b, double D[3]) {
    double ca = a - 0.5 * (nu - 1), cb = b - 0.5 * (nv - 1);
    for (int k = 0; k < 3; ++k) {
        double q = view[3 + k] + ca * view[6 + k] + cb * view[9 + k];
        D[k] = q - view[k];
    }
}

static bool view_separable(const double *v) {
    // detector columns horizontal (u_z = 0) and rows along z (v_x = v_y = 0)
    return v[8] == 0.0 && v[9] == 0.0 && v[10] == 0.0;
}

int check_geometry(int nx, int ny, int nz, double h, const double *origin, int nu, int nv, int nviews,
                   const double *views) {
    if (nx < 1 || ny < 1 || nz < 1 || nu < 1 || nv < 1 || nviews < 1) return MGCT_ERR_INVALID_ARG;
    if (!(h > 0.0) || !isfinite(h) || !origin || !views) return MGCT_ERR_INVALID_ARG;
    if ((double)nx * ny * nz > 2.0e9 || (double)nviews * nu * nv > 4.0e9) return MGCT_ERR_INVALID_ARG;
    int n[3] = {nx, ny, nz};
    for (int v = 0; v < nviews; ++v) {
        const double *w = views + (size_t)v * 12;
        for (int k = 0; k < 12; ++k)
            if (!isfinite(w[k])) return MGCT_ERR_INVALID_ARG;
        // source at least one voxel outside the box [-0.5, n-0.5] (index units)
        bool inside = true;
        for (int k = 0; k < 3; ++k) {
            double si = (w[k] - origin[k]) / h + 0.5 * (n[k] - 1);
            if (si < -1.5 || si > n[k] + 0.5) inside = false;
        }
        if (inside) return MGCT_ERR_UNSUPPORTED_GEOMETRY;
        // u and v must span a plane
        double cx = w[7] * w[11] - w[8] * w[10], cy = w[8] * w[9] - w[6] * w[11], cz = w[6] * w[10] - w[7] * w[9];
        if (cx == 0.0 && cy == 0.0 && cz == 0.0) return MGCT_ERR_INVALID_ARG;
    }
    return MGCT_OK;
}

int build_level(Ctx &c, int g, Level &L) {
    const int f = 1 << g;
    if (c.nx % f || c.ny % f || c.nz % f || c.nu % f || c.nv % f) return MGCT_ERR_SIZE_NOT_DIVISIBLE;
    L.nx = c.nx / f;
    L.ny = c.ny / f;
    L.nz = c.nz / f;
    L.nu = c.nu / f;
    L.nv = c.nv / f;
    L.nviews = c.nviews;
    L.h = c.h * f;
    const int V = L.nviews, nu = L.nu, nv = L.nv;
    const int n[3] = {L.nx, L.ny, L.nz};

    // physical views of this level: same s and d, steps scaled by 2^g (exact)
    std::vector<double> pv(c.views);
    bool sep = true;
    for (int v = 0; v < V; ++v) {
        double *w = &pv[(size_t)v * 12];
        for (int k = 6; k < 12; ++k) w[k] *= f;
        sep = sep && view_separable(w);
    }
    L.separable = sep;

    std::vector<ViewIdx> vi(V);
    for (int v = 0; v < V; ++v) {
        const double *w = &pv[(size_t)v * 12];
        for (int k = 0; k < 3; ++k) {
            double cc = 0.5 * (n[k] - 1);
            vi[v].s[k] = (w[k] - c.origin[k]) / L.h + cc;
            vi[v].d[k] = (w[3 + k] - c.origin[k]) / L.h + cc;
            vi[v].u[k] = w[6 + k] / L.h;
            vi[v].v[k] = w[9 + k] / L.h;
        }
    }

    // major-axis table
    std::vector<uint8_t> axis;
    if (sep) {
        axis.resize((size_t)V * nu);
        for (int v = 0; v < V; ++v) {
            const double *w = &pv[(size_t)v * 12];
            for (int a = 0; a < nu; ++a) {
                double D0[3], D1[3];
                ray_dir(w, nu, nv, a, 0, D0);
                ray_dir(w, nu, nv, a, nv - 1, D1);
                int m0 = major_axis_phys(D0), m1 = major_axis_phys(D1);
                // |D_z| is largest at an end row, and D_x, D_y do not depend on
                // the row, so checking both end rows finds every z-major ray.
                if (m0 == 2 || m1 == 2) return MGCT_ERR_UNSUPPORTED_GEOMETRY;
                axis[(size_t)v * nu + a] = (uint8_t)m0;
            }
        }
        L.axis_row_stride = 0;
    } else {
        axis.resize((size_t)V * nu * nv);
        for (int v = 0; v < V; ++v) {
            const double *w = &pv[(size_t)v * 12];
            for (int b = 0; b < nv; ++b)
                for (int a = 0; a < nu; ++a) {
                    double D[3];
                    ray_dir(w, nu, nv, a, b, D);
                    int m = major_axis_phys(D);
                    if (m == 2) return MGCT_ERR_UNSUPPORTED_GEOMETRY;
                    axis[((size_t)v * nv + b) * nu + a] = (uint8_t)m;
                }
        }
        L.axis_row_stride = nu;
    }

    std::vector<SepView> sv;
    std::vector<ColD> cols;
    if (sep) {
        sv.resize(V);
        cols.resize((size_t)V * nu);
        for (int v = 0; v < V; ++v) {
            const ViewIdx &q = vi[v];
            SepView &o = sv[v];
            o.sx = q.s[0];
            o.sy = q.s[1];
            o.sz = q.s[2];
            o.dz0 = q.d[2] - 0.5 * (nv - 1) * q.v[2] - q.s[2];
            o.vz = q.v[2];
            // column hit by the ray from s through (px, py): with e = s - d and
            // w = P - s, alpha = (e x w) / (u x w) (2-D cross products), and
            // a = alpha + (nu-1)/2.  Written as a ratio of affine functions of P.
            double ex = q.s[0] - q.d[0], ey = q.s[1] - q.d[1];
            double ux = q.u[0], uy = q.u[1];
            double an1 = -ey, an2 = ex, an0 = ey * q.s[0] - ex * q.s[1];
            double ad1 = -uy, ad2 = ux, ad0 = uy * q.s[0] - ux * q.s[1];
            double cu = 0.5 * (nu - 1);
            o.an0 = (float)(an0 + cu * ad0);
            o.an1 = (float)(an1 + cu * ad1);
            o.an2 = (float)(an2 + cu * ad2);
            o.ad0 = (float)ad0;
            o.ad1 = (float)ad1;
            o.ad2 = (float)ad2;
            o.flags = 0;
            o.pad = 0;
            o.r0lo = o.r1lo = HUGE_VAL;
            o.r0hi = o.r1hi = -HUGE_VAL;
            for (int a = 0; a < nu; ++a) {
                double ca = a - 0.5 * (nu - 1);
                double Dx = q.d[0] + ca * q.u[0] - q.s[0];
                double Dy = q.d[1] + ca * q.u[1] - q.s[1];
                cols[(size_t)v * nu + a] = ColD{Dx, Dy, 1.0 / Dx, 1.0 / Dy, Dx / q.v[2], Dy / q.v[2],
                                                (int)axis[(size_t)v * nu + a], {0, 0, 0}};
                o.flags |= axis[(size_t)v * nu + a] == 0 ? 1 : 2;
                if (axis[(size_t)v * nu + a] == 0) {
                    o.r0lo = std::min(o.r0lo, 1.0 / Dx);
                    o.r0hi = std::max(o.r0hi, 1.0 / Dx);
                } else {
                    o.r1lo = std::min(o.r1lo, 1.0 / Dy);
                    o.r1hi = std::max(o.r1hi, 1.0 / Dy);
                }
            }
        }
    }

    // The LDS projector's block order: (view, row tile) pairs with the views
    // grouped by source height (one row tile of views at one height samples
    // one z band of the volume), groups by height, views by angle within one.
    std::vector<int> order;
    if (sep) {
        L.n_rt = (nv + 63) / 64;
        std::vector<int> idx(V);
        for (int v = 0; v < V; ++v) idx[v] = v;
        const double cx = 0.5 * (L.nx - 1), cy = 0.5 * (L.ny - 1);
        std::stable_sort(idx.begin(), idx.end(), [&](int p, int q) {
            if (vi[p].s[2] != vi[q].s[2]) return vi[p].s[2] < vi[q].s[2];
            return atan2(vi[p].s[1] - cy, vi[p].s[0] - cx) < atan2(vi[q].s[1] - cy, vi[q].s[0] - cx);
        });
        order.reserve((size_t)V * L.n_rt);
        for (int g0 = 0; g0 < V;) {
            int g1 = g0 + 1;
            while (g1 < V && vi[idx[g1]].s[2] == vi[idx[g0]].s[2]) ++g1;
            for (int r = 0; r < L.n_rt; ++r)
                for (int k = g0; k < g1; ++k) order.push_back(idx[k] * L.n_rt + r);
            g0 = g1;
        }
    }

    // upload
    if (hipMalloc(&L.d_views, sizeof(ViewIdx) * V) != hipSuccess) return MGCT_ERR_OOM;
    if (hipMemcpy(L.d_views, vi.data(), sizeof(ViewIdx) * V, hipMemcpyHostToDevice) != hipSuccess)
        return MGCT_ERR_HIP;
    if (hipMalloc(&L.d_axis, axis.size()) != hipSuccess) return MGCT_ERR_OOM;
    if (hipMemcpy(L.d_axis, axis.data(), axis.size(), hipMemcpyHostToDevice) != hipSuccess) return MGCT_ERR_HIP;
    if (sep) {
        if (hipMalloc(&L.d_sep, sizeof(SepView) * V) != hipSuccess) return MGCT_ERR_OOM;
        if (hipMemcpy(L.d_sep, sv.data(), sizeof(SepView) * V, hipMemcpyHostToDevice) != hipSuccess)
            return MGCT_ERR_HIP;
        if (hipMalloc(&L.d_cols, sizeof(ColD) * cols.size()) != hipSuccess) return MGCT_ERR_OOM;
        if (hipMemcpy(L.d_cols, cols.data(), sizeof(ColD) * cols.size(), hipMemcpyHostToDevice) != hipSuccess)
            return MGCT_ERR_HIP;
        if ((double)V * L.n_rt < 2.0e9) {
            if (hipMalloc(&L.d_order, sizeof(int) * order.size()) != hipSuccess) return MGCT_ERR_OOM;
            if (hipMemcpy(L.d_order, order.data(), sizeof(int) * order.size(), hipMemcpyHostToDevice) != hipSuccess)
                return MGCT_ERR_HIP;
            // the learned step's judge: every judge_step-th view (about 360
            // views) once a scan has 720 views or more, in the same order
            L.judge_step = V >= 720 ? V / 360 : 1;
            if (L.judge_step > 1) {
                std::vector<int> jo;
                for (int e : order)
                    if ((e / L.n_rt) % L.judge_step == 0) jo.push_back(e);
                L.n_t_judge = (int)jo.size();
                if (hipMalloc(&L.d_order_judge, sizeof(int) * jo.size()) != hipSuccess) return MGCT_ERR_OOM;
                if (hipMemcpy(L.d_order_judge, jo.data(), sizeof(int) * jo.size(), hipMemcpyHostToDevice) !=
                    hipSuccess)
                    return MGCT_ERR_HIP;
            }
        }
    }
    return MGCT_OK;
}

void free_level(Level &L) {
    if (L.d_views) (void)hipFree(L.d_views);
    if (L.d_sep) (void)hipFree(L.d_sep);
    if (L.d_cols) (void)hipFree(L.d_cols);
    if (L.d_axis) (void)hipFree(L.d_axis);
    if (L.d_order) (void)hipFree(L.d_order);
    if (L.d_order_judge) (void)hipFree(L.d_order_judge);
    L.d_order = nullptr;
    L.d_order_judge = nullptr;
    L.judge_step = 1;
    L.n_t_judge = 0;
    L.d_views = nullptr;
    L.d_sep = nullptr;
    L.d_cols = nullptr;
    L.d_axis = nullptr;
}

}  // namespace mgct
