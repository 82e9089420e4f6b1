// Host-only part of the C ABI: argument validation, grid metrics, eigenvalue
// and twiddle tables, workspace layout.  Contains no HIP call, so a plan can
// be created and inspected on a machine without a GPU.
#include "fsei_plan.h"

#include <cmath>
#include <algorithm>
#include <cstring>
#include <new>

namespace fsei {

static const long double kPi = 3.141592653589793238462643383279502884L;

bool factor_radices(int n, FftPlan* out) {
    FftPlan p;
    p.n = n;
    int m = n;
    int r3 = 0;
    while (m % 3 == 0) { m /= 3; ++r3; }
    // m is now a power of two (or the size was rejected by the caller)
    if (m & (m - 1)) return false;
    while (m >= 8 && (m % 8) == 0) { p.radix[p.nstages++] = 8; m /= 8; }
    if (m == 4) { p.radix[p.nstages++] = 4; m = 1; }
    if (m == 2) { p.radix[p.nstages++] = 2; m = 1; }
    for (int i = 0; i < r3; ++i) p.radix[p.nstages++] = 3;
    if (p.nstages > kMaxStages) return false;
    *out = p;
    return true;
}

static bool valid_xy(int n) {
    if (n < 2 || n > kMaxN) return false;
    int m = n;
    while (m % 2 == 0) m /= 2;
    while (m % 3 == 0) m /= 3;
    return m == 1;
}

static size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

void compute_layout(fsei_plan_impl* p) {
    const size_t N = p->ncells();
    // FP32 plans route the near-singular lowest-mode lines to FP64:
    // kappa = 1 + 4 / (dz_min^2 |sigma|) > kappa_star
    p->list_host.clear();
    p->sigma_thr = 0.0;
    if (p->precision != FSEI_PREC_FP64) {
        p->sigma_thr = 4.0 / (p->dzmin * p->dzmin * (p->kappa_star - 1.0));
        const double* lx = p->tab_d.data() + p->tab_off[T_LAMX];
        const double* ly = p->tab_d.data() + p->tab_off[T_LAMY];
        for (int qy = 0; qy < p->ny; ++qy)
            for (int qx = 0; qx < p->nx; ++qx) {
                if (qx == 0 && qy == 0) continue;
                if (std::fabs(lx[qx] + ly[qy]) < p->sigma_thr) p->list_host.push_back(qy * p->nx + qx);
            }
    }
    p->nlist = (int)p->list_host.size();
    const long nseq = x_nseq(p->nx);
    // one partial triple per x-forward tile, or per 8-row tile of the
    // residual-norm pass, whichever is more
    p->n_partials = (size_t)std::max(((long)p->ny * p->nz + 2 * nseq - 1) / (2 * nseq),
                                     (long)((p->ny + 7) / 8) * p->nz);

    size_t off = 0;
    p->ws_tab_d = off;
    off = round_up(off + p->tab_elems * sizeof(double), kAlign);
    p->ws_tab_f = off;
    off = round_up(off + p->tab_elems * sizeof(float), kAlign);
    p->ws_scalars = off;
    off = round_up(off + fsei_plan_impl::kScalars * sizeof(double), kAlign);
    p->ws_partials = off;
    off = round_up(off + 3 * (p->n_partials + kSumGroups) * sizeof(double), kAlign);   // + group sums
    p->ws_list = off;
    p->ws_list_bytes = (size_t)p->nlist * sizeof(int);
    off = round_up(off + p->ws_list_bytes, kAlign);
    // field 1: the intermediate field (FP64; FP32 for FP32 plans); for
    // FP32_REFINE it keeps f = D u* / dt in FP64
    const size_t esz = (p->precision == FSEI_PREC_FP32) ? sizeof(float) : sizeof(double);
    p->ws_field = off;
    p->ws_field_bytes = N * esz;
    off = round_up(off + p->ws_field_bytes, kAlign);
    // FP32_REFINE: FP32 correction field and an FP64 pressure field
    const bool refine = p->precision == FSEI_PREC_FP32_REFINE;
    p->ws_field2 = off;
    p->ws_field2_bytes = refine ? N * sizeof(float) : 0;
    off = round_up(off + p->ws_field2_bytes, kAlign);
    p->ws_field3 = off;
    p->ws_field3_bytes = refine ? N * sizeof(double) : 0;
    off = round_up(off + p->ws_field3_bytes, kAlign);
    p->ws_field4 = off;
    p->ws_field4_bytes = refine ? N * sizeof(float) : 0;
    off = round_up(off + p->ws_field4_bytes, kAlign);
    p->ws_total = off;
}

static void build_tables(fsei_plan_impl* p) {
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    size_t len[T_COUNT];
    for (int t = T_ZA; t <= T_GAM_ADJ; ++t) len[t] = nz;
    len[T_LAMX] = nx;
    len[T_LAMY] = ny;
    len[T_TWX_C] = len[T_TWX_S] = len[T_DCTX_C] = len[T_DCTX_S] = nx;
    len[T_TWY_C] = len[T_TWY_S] = len[T_DCTY_C] = len[T_DCTY_S] = ny;
    size_t off = 0;
    for (int t = 0; t < T_COUNT; ++t) {
        p->tab_off[t] = off;
        off += (len[t] + 31) / 32 * 32;   // keep every table 256-B aligned in double
    }
    p->tab_elems = off;
    std::vector<long double> tab(off, 0.0L);
    auto T = [&](int id) { return tab.data() + p->tab_off[id]; };

    // z metrics in long double from the caller's face coordinates
    std::vector<long double> dz(nz), zm(nz), h(nz, 0.0L);
    for (int k = 0; k < nz; ++k) {
        dz[k] = (long double)p->zc[k + 1] - (long double)p->zc[k];
        zm[k] = 0.5L * ((long double)p->zc[k] + (long double)p->zc[k + 1]);
    }
    for (int k = 1; k < nz; ++k) h[k] = zm[k] - zm[k - 1];
    for (int k = 0; k < nz; ++k) {
        long double a = (k >= 1) ? 1.0L / (dz[k] * h[k]) : 0.0L;
        long double c = (k <= nz - 2) ? 1.0L / (dz[k] * h[k + 1]) : 0.0L;
        T(T_ZA)[k] = a;
        T(T_ZC)[k] = c;
        T(T_ZB0)[k] = -(a + c);
        T(T_DZ)[k] = dz[k];
        T(T_INV_DZ)[k] = 1.0L / dz[k];
        T(T_INV_H)[k] = (k >= 1) ? 1.0L / h[k] : 0.0L;
        T(T_H)[k] = h[k];
        T(T_ZETA_ADJ)[k] = (k <= nz - 2) ? 1.0L / h[k + 1] : 0.0L;
        T(T_GAM_ADJ)[k] = (k >= 1) ? 1.0L / dz[k - 1] : 0.0L;
    }
    // modified wavenumbers of the 3-point second difference on each
    // transform row: DCT-II row q -> wavenumber q; half-complex row q ->
    // min(q, n-q)
    auto lam = [](int n, double d, int bc, long double* out) {
        for (int q = 0; q < n; ++q) {
            long double arg;
            if (bc == FSEI_BC_WALL) {
                arg = kPi * q / (2.0L * n);
            } else {
                int m = (q <= n - q) ? q : n - q;
                arg = kPi * m / (long double)n;
            }
            long double s = sinl(arg);
            out[q] = -4.0L / ((long double)d * (long double)d) * s * s;
        }
    };
    lam(nx, p->dx, p->bcx, T(T_LAMX));
    lam(ny, p->dy, p->bcy, T(T_LAMY));
    auto tw = [](int n, long double* c, long double* s, long double* dc, long double* ds) {
        for (int t = 0; t < n; ++t) {
            c[t] = cosl(2.0L * kPi * t / n);
            s[t] = sinl(2.0L * kPi * t / n);
            dc[t] = cosl(kPi * t / (2.0L * n));
            ds[t] = sinl(kPi * t / (2.0L * n));
        }
    };
    tw(nx, T(T_TWX_C), T(T_TWX_S), T(T_DCTX_C), T(T_DCTX_S));
    tw(ny, T(T_TWY_C), T(T_TWY_S), T(T_DCTY_C), T(T_DCTY_S));

    p->tab_d.assign(off, 0.0);
    p->tab_f.assign(off, 0.0f);
    for (size_t i = 0; i < off; ++i) {
        p->tab_d[i] = (double)tab[i];
        p->tab_f[i] = (float)tab[i];
    }
    p->dz.assign(nz, 0.0);
    p->h.assign(nz, 0.0);
    long double lz = 0.0L;
    double dzmin = 1e300;
    for (int k = 0; k < nz; ++k) {
        p->dz[k] = (double)dz[k];
        p->h[k] = (double)h[k];
        lz += dz[k];
        if (p->dz[k] < dzmin) dzmin = p->dz[k];
    }
    p->lz = (double)lz;
    p->dzmin = dzmin;
}

}  // namespace fsei

using namespace fsei;

extern "C" {

const char* fsei_status_string(fsei_status s) {
    switch (s) {
        case FSEI_OK: return "FSEI_OK";
        case FSEI_ERR_ARG: return "FSEI_ERR_ARG: invalid argument";
        case FSEI_ERR_SIZE: return "FSEI_ERR_SIZE: unsupported grid size";
        case FSEI_ERR_GRID: return "FSEI_ERR_GRID: invalid grid metrics";
        case FSEI_ERR_WORKSPACE: return "FSEI_ERR_WORKSPACE: workspace missing, too small or misaligned";
        case FSEI_ERR_HIP: return "FSEI_ERR_HIP: HIP runtime error";
        case FSEI_ERR_NOT_CONVERGED: return "FSEI_ERR_NOT_CONVERGED: refinement did not reach rtol";
        case FSEI_ERR_PRECISION: return "FSEI_ERR_PRECISION: entry point does not match the plan precision";
    }
    return "unknown fsei_status";
}

fsei_status fsei_poisson_plan_create(int nx, int ny, int nz, const int bc[2], double dx, double dy,
                                     const double* zc, fsei_plan** out) {
    if (!out) return FSEI_ERR_ARG;
    *out = nullptr;
    if (!bc || !zc) return FSEI_ERR_ARG;
    for (int d = 0; d < 2; ++d)
        if (bc[d] != FSEI_BC_PERIODIC && bc[d] != FSEI_BC_WALL) return FSEI_ERR_ARG;
    if (!valid_xy(nx) || !valid_xy(ny)) return FSEI_ERR_SIZE;
    if (nz < 2 || nz > kMaxNz) return FSEI_ERR_SIZE;
    if (!(std::isfinite(dx) && std::isfinite(dy)) || dx <= 0.0 || dy <= 0.0) return FSEI_ERR_GRID;
    for (int k = 0; k <= nz; ++k)
        if (!std::isfinite(zc[k])) return FSEI_ERR_GRID;
    for (int k = 0; k < nz; ++k)
        if (!(zc[k + 1] > zc[k])) return FSEI_ERR_GRID;
    fsei_plan* p = new (std::nothrow) fsei_plan();
    if (!p) return FSEI_ERR_ARG;
    p->nx = nx;
    p->ny = ny;
    p->nz = nz;
    p->bcx = bc[0];
    p->bcy = bc[1];
    p->dx = dx;
    p->dy = dy;
    p->zc.assign(zc, zc + nz + 1);
    if (!factor_radices(nx, &p->fx) || !factor_radices(ny, &p->fy)) {
        delete p;
        return FSEI_ERR_SIZE;
    }
    build_tables(p);
    compute_layout(p);
    *out = p;
    return FSEI_OK;
}

fsei_status fsei_plan_set_precision(fsei_plan* p, int precision, double rtol, int max_iter) {
    if (!p) return FSEI_ERR_ARG;
    if (precision != FSEI_PREC_FP64 && precision != FSEI_PREC_FP32_REFINE && precision != FSEI_PREC_FP32)
        return FSEI_ERR_ARG;
    if (!std::isfinite(rtol) || rtol < 0.0 || max_iter < 0 || max_iter > 64) return FSEI_ERR_ARG;
    p->precision = precision;
    p->rtol = rtol;
    p->max_iter = max_iter;
    compute_layout(p);
    // the layout changed: the caller sets a workspace again
    p->ws = nullptr;
    p->ws_bytes = 0;
    return FSEI_OK;
}

fsei_status fsei_plan_workspace_size(const fsei_plan* p, size_t* bytes) {
    if (!p || !bytes) return FSEI_ERR_ARG;
    *bytes = p->ws_total;
    return FSEI_OK;
}

}  // extern "C"
