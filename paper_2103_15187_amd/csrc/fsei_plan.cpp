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
    // The near-singular lowest-mode lines, kappa = 1 + 4 / (dz_min^2 |sigma|)
    // > kappa_star, are solved one per lane in FP64 with row-sum pivots (in
    // every precision mode); the tiled solvers skip them.
    p->list_host.clear();
    p->sigma_thr = 4.0 / (p->dzmin * p->dzmin * (p->kappa_star - 1.0));
    {
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
    // FP64 scratch of the near-singular lines: eliminated right-hand side and
    // c_k / d_k, nlist * nz each
    p->ws_seq = off;
    off = round_up(off + 2 * (size_t)p->nlist * (size_t)p->nz * sizeof(double), kAlign);
    // viscous line-solve tables (3 components x 3 directions)
    p->visc_L[0] = visc_chunk(p->nx);
    p->visc_L[1] = visc_chunk(p->ny);
    p->visc_L[2] = visc_chunk(p->nz);
    p->ws_visc = off;
    p->ws_visc_comp = 0;
    if (p->visc_L[0] && p->visc_L[1] && p->visc_L[2])
        p->ws_visc_comp = round_up((size_t)(visc_tab_elems(p->visc_L[0]) + visc_tab_elems(p->visc_L[1]) +
                                            visc_tab_elems(p->visc_L[2])) * sizeof(double), kAlign);
    off = round_up(off + 3 * p->ws_visc_comp, kAlign);
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
    for (int t = T_ZA; t <= T_HF; ++t) len[t] = nz;
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
        T(T_ZF)[k] = p->zc[k];
        T(T_ZM)[k] = zm[k];
        T(T_HF)[k] = (k >= 1) ? h[k] : 0.5L * dz[0];
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
        case FSEI_ERR_SCRATCH: return "FSEI_ERR_SCRATCH: the plan's workspace exceeds the allocation-free scratch";
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

// ---------------------------------------------------------------------------
// Viscous line-solve tables (paper, Sec. 2.1 eq. NSdiscr0 and Sec. 3: the
// Crank-Nicolson viscous operator, approximately factorised into one
// tridiagonal matrix I - beta L_d per direction, Thomas' algorithm with a
// Sherman-Morrison correction for periodic lines).
//
// L_d is the staggered three-point second difference of the component:
// along its own axis the component lives on faces (walls: the stored wall
// face is dead, the opposite wall face is zero); along the other axes at
// cell centres (walls: no-slip through a mirrored ghost, a wall flux of
// 2 q / spacing over the half cell).  z is stretched and walled.
// ---------------------------------------------------------------------------
namespace fsei {

namespace {

struct Tri {
    std::vector<double> a, b, c;   // sub, diagonal, super of I - beta L
    double corner_lo = 0.0;        // periodic: entry (0, n-1)
    double corner_hi = 0.0;        // periodic: entry (n-1, 0)
    bool cyc = false;
    bool dead0 = false;            // row 0 is a dead wall face
};

Tri visc_matrix(const fsei_plan_impl* p, int comp, int dir, double beta) {
    Tri m;
    const bool own = comp == dir;
    const int n = dir == 0 ? p->nx : dir == 1 ? p->ny : p->nz;
    m.a.assign(n, 0.0);
    m.b.assign(n, 1.0);
    m.c.assign(n, 0.0);
    if (dir < 2) {
        const double d = dir == 0 ? p->dx : p->dy;
        const int bc = dir == 0 ? p->bcx : p->bcy;
        const double k2 = beta / (d * d);
        for (int i = 0; i < n; ++i) {
            m.a[i] = (i > 0) ? -k2 : 0.0;
            m.c[i] = (i + 1 < n) ? -k2 : 0.0;
            m.b[i] = 1.0 + 2.0 * k2;
        }
        if (bc == FSEI_BC_PERIODIC) {
            m.cyc = true;
            m.corner_lo = -k2;
            m.corner_hi = -k2;
        } else if (own) {
            // face 0 is the wall (dead); the face beyond the last is the
            // other wall, value 0: the last row just loses its coupling
            m.dead0 = true;
            m.b[0] = 1.0;
            m.c[0] = 0.0;
            if (n > 1) m.a[1] = 0.0;
        } else {
            // mirrored ghost at both walls
            m.b[0] = 1.0 + 3.0 * k2;
            m.b[n - 1] = 1.0 + 3.0 * k2;
        }
        return m;
    }
    const std::vector<double>& dz = p->dz;
    const std::vector<double>& h = p->h;
    if (own) {
        // w on z faces: face 0 is the bottom wall (dead), face nz the top wall
        m.dead0 = true;
        for (int k = 1; k < n; ++k) {
            const double lo = 1.0 / (dz[k - 1] * h[k]);
            const double hi = 1.0 / (dz[k] * h[k]);
            m.a[k] = (k - 1 >= 1) ? -beta * lo : 0.0;
            m.c[k] = (k + 1 < n) ? -beta * hi : 0.0;
            m.b[k] = 1.0 + beta * (lo + hi);
        }
        return m;
    }
    for (int k = 0; k < n; ++k) {
        const double lo = (k >= 1) ? 1.0 / (h[k] * dz[k]) : 2.0 / (dz[0] * dz[0]);
        const double hi = (k + 1 < n) ? 1.0 / (h[k + 1] * dz[k]) : 2.0 / (dz[k] * dz[k]);
        m.a[k] = (k >= 1) ? -beta * lo : 0.0;
        m.c[k] = (k + 1 < n) ? -beta * hi : 0.0;
        m.b[k] = 1.0 + beta * (lo + hi);
    }
    return m;
}

// Thomas solve on the host (periodic Sherman-Morrison vector only)
std::vector<double> host_thomas(const std::vector<double>& a, const std::vector<double>& b,
                                const std::vector<double>& c, std::vector<double> f) {
    const int n = (int)b.size();
    std::vector<double> cp(n);
    double piv = b[0];
    cp[0] = c[0] / piv;
    f[0] /= piv;
    for (int i = 1; i < n; ++i) {
        piv = b[i] - a[i] * cp[i - 1];
        cp[i] = c[i] / piv;
        f[i] = (f[i] - a[i] * f[i - 1]) / piv;
    }
    for (int i = n - 2; i >= 0; --i) f[i] -= cp[i] * f[i + 1];
    return f;
}

void visc_block(const Tri& m0, int L, double* out) {
    const int n = (int)m0.b.size();
    const int NP = kViscPmax * L;
    double* rr = out;
    double* al = out + NP;
    double* wr = out + 2 * NP;
    double* cn = out + 3 * NP;
    double* vr = out + 4 * NP;
    double* zt = out + 5 * NP;
    double* wl = out + 6 * NP;
    double* vl = wl + kViscLv * kViscPmax;
    std::fill(out, out + visc_tab_elems(L), 0.0);
    Tri m = m0;
    double vq = 0.0;
    if (m.cyc) {
        // A = A' + u v^T with u = (g, 0, .., corner_hi), v = (1, 0, .., corner_lo / g)
        const double g = -m.b[0];
        m.b[0] -= g;
        m.b[n - 1] -= m.corner_lo * m.corner_hi / g;
        vq = m.corner_lo / g;
        std::vector<double> u(n, 0.0);
        u[0] = g;
        u[n - 1] += m.corner_hi;
        const std::vector<double> z = host_thomas(m.a, m.b, m.c, u);
        const double den = 1.0 + z[0] + vq * z[n - 1];
        for (int t = 0; t < n; ++t) zt[t] = z[t] / den;
    }
    // Thomas factorisation of the (modified) tridiagonal matrix: pivots,
    // then the coefficients of the two substitution recurrences
    std::vector<double> pv(n);
    pv[0] = m.b[0];
    for (int t = 1; t < n; ++t) pv[t] = m.b[t] - m.a[t] * m.c[t - 1] / pv[t - 1];
    for (int t = 0; t < n; ++t) {
        rr[t] = (t == 0 && m.dead0) ? 0.0 : 1.0 / pv[t];
        al[t] = (t == 0) ? 0.0 : -m.a[t] * rr[t];
        cn[t] = -m.c[t] * rr[t];
    }
    // per-row carry products inside each chunk
    for (int q = 0; q < kViscPmax; ++q) {
        double pr = 1.0;
        for (int t = q * L; t < (q + 1) * L; ++t) {
            pr *= al[t];
            wr[t] = pr;
        }
        pr = 1.0;
        for (int t = (q + 1) * L - 1; t >= q * L; --t) {
            pr *= cn[t];
            vr[t] = pr;
        }
    }
    // Kogge-Stone multipliers over the chunks
    double W[kViscPmax], Vv[kViscPmax];
    for (int q = 0; q < kViscPmax; ++q) {
        W[q] = wr[q * L + L - 1];
        Vv[q] = vr[q * L];
    }
    for (int lv = 0; lv < kViscLv; ++lv) {
        const int s = 1 << lv;
        double Wn[kViscPmax], Vn[kViscPmax];
        for (int q = 0; q < kViscPmax; ++q) {
            wl[lv * kViscPmax + q] = W[q];
            vl[lv * kViscPmax + q] = Vv[q];
            Wn[q] = (q >= s) ? W[q] * W[q - s] : W[q];
            Vn[q] = (q + s < kViscPmax) ? Vv[q] * Vv[q + s] : Vv[q];
        }
        for (int q = 0; q < kViscPmax; ++q) {
            W[q] = Wn[q];
            Vv[q] = Vn[q];
        }
    }
    vl[kViscLv * kViscPmax] = vq;
}

}  // namespace

void build_visc_tables(const fsei_plan_impl* p, int comp, double beta, double* out) {
    for (int d = 0; d < 3; ++d) {
        const int L = p->visc_L[d];
        visc_block(visc_matrix(p, comp, d, beta), L, out);
        out += visc_tab_elems(L);
    }
}

}  // namespace fsei
