// fsei_momentum.h -- explicit right-hand side of the momentum step.
//
// Paper, Sec. 2.1, eq. NSdiscr0: Adams-Bashforth (weights gamma, rho) for
// the convective term, Crank-Nicolson for the viscous term; with the pressure
// left to the projection, the increment du = u* - u^n of the provisional
// velocity solves (I - beta Lap) du = rhs with
//
//     rhs = dt [ -(gamma N^n + rho N^{n-1}) + (1/Re) Lap u^n ],   N = div(u u).
//
// N is the divergence form on each component's control volume of the
// staggered grid: fluxes of momentum are products of two-point means (x, y)
// and of linear z interpolations (stretched z), walls carry no flux (zero
// normal velocity); Lap is the component's three-point operator of the
// implicit viscous step (faces along its own axis with Dirichlet walls,
// centres along the others with a mirrored no-slip ghost).
#pragma once

#include <hip/hip_runtime.h>

#include "fsei_plan.h"
#include "fsei_transforms.h"   // xcd_remap

namespace fsei {
namespace dev {

struct MomArgs {
    int nx, ny, nz, perx, pery;
    const double* u;
    const double* v;
    const double* w;
    double* nu;   // in: N^{n-1} (read when rho != 0); out: N^n
    double* nv;
    double* nw;
    double* ru;   // out: right-hand sides
    double* rv;
    double* rw;
    double idx, idy, idx2, idy2;
    double dt, inv_re, gamma, rho;
    const double* dz;       // dz_k
    const double* inv_dz;   // 1/dz_k
    const double* inv_h;    // 1/h_k (k >= 1)
    const double* za;       // 1/(dz_k h_k), k >= 1
    const double* zc;       // 1/(dz_k h_{k+1}), k <= nz-2
};

// One workgroup per (j, k) row; lanes over x.  Rows are visited in tiles
// of GJ rows, plane by plane inside a tile, each XCD taking a contiguous run
// of rows: the j +- 1 and k +- 1 rows a workgroup reads were just read by its
// neighbours on the same XCD (L2 hits rather than HBM re-reads).
template <int NT, int GJ>
__global__ __launch_bounds__(NT) void k_momentum_rhs(MomArgs a) {
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int b = (int)xcd_remap(blockIdx.x, gridDim.x);
    const int per = nz * GJ;
    const int jt = b / per;
    const int rem = b - jt * per;
    const int k = rem / GJ;
    const int j = jt * GJ + (rem - k * GJ);
    const size_t nxy = (size_t)nx * ny;
    const bool wx = !a.perx, wy = !a.pery;
    // field value with the grid's boundary conventions: outside the grid 0
    // (walls) or wrapped (periodic); dead wall faces read as 0
    auto U = [&](int i, int jj, int kk) -> double {
        if (kk < 0 || kk >= nz) return 0.0;
        if (i < 0 || i >= nx) {
            if (wx) return 0.0;
            i = (i + nx) % nx;
        }
        if (jj < 0 || jj >= ny) {
            if (wy) return 0.0;
            jj = (jj + ny) % ny;
        }
        if (wx && i == 0) return 0.0;
        return a.u[(size_t)kk * nxy + (size_t)jj * nx + i];
    };
    auto Vv = [&](int i, int jj, int kk) -> double {
        if (kk < 0 || kk >= nz) return 0.0;
        if (i < 0 || i >= nx) {
            if (wx) return 0.0;
            i = (i + nx) % nx;
        }
        if (jj < 0 || jj >= ny) {
            if (wy) return 0.0;
            jj = (jj + ny) % ny;
        }
        if (wy && jj == 0) return 0.0;
        return a.v[(size_t)kk * nxy + (size_t)jj * nx + i];
    };
    auto Ww = [&](int i, int jj, int kk) -> double {
        if (kk <= 0 || kk >= nz) return 0.0;   // face 0 is the bottom wall, nz the top
        if (i < 0 || i >= nx) {
            if (wx) return 0.0;
            i = (i + nx) % nx;
        }
        if (jj < 0 || jj >= ny) {
            if (wy) return 0.0;
            jj = (jj + ny) % ny;
        }
        return a.w[(size_t)kk * nxy + (size_t)jj * nx + i];
    };
    // z interpolation weights to faces k and k+1 (weight of the lower centre,
    // of the upper centre); face 0 and face nz carry no flux
    const double dzk = a.dz[k];
    const double wlo0 = (k >= 1) ? dzk / (a.dz[k - 1] + dzk) : 0.0;
    const double whi0 = (k >= 1) ? a.dz[k - 1] / (a.dz[k - 1] + dzk) : 0.0;
    const double wlo1 = (k + 1 < nz) ? a.dz[k + 1] / (dzk + a.dz[k + 1]) : 0.0;
    const double whi1 = (k + 1 < nz) ? dzk / (dzk + a.dz[k + 1]) : 0.0;
    const double idz = a.inv_dz[k];
    const double ihk = (k >= 1) ? a.inv_h[k] : 0.0;
    // z Laplacian coefficients: centres (u, v) and faces (w)
    const double clo = (k >= 1) ? a.za[k] : 2.0 * idz * idz;
    const double chi = (k + 1 < nz) ? a.zc[k] : 2.0 * idz * idz;
    const double flo = (k >= 2) ? a.inv_dz[k - 1] * ihk : 0.0;        // w_{k-1} live only for k-1 >= 1
    const double fhi = (k + 1 < nz) ? idz * ihk : 0.0;
    const double fdg = (k >= 1) ? (a.inv_dz[k - 1] + idz) * ihk : 0.0;   // both neighbours' weights
    const size_t row = (size_t)k * nxy + (size_t)j * nx;
    for (int i = threadIdx.x; i < nx; i += NT) {
        const size_t o = row + i;
        // ---------------- u at x-face i
        double ru = 0.0, nun = 0.0;
        if (!(wx && i == 0)) {
            const double u0 = U(i, j, k), uxp = U(i + 1, j, k), uxm = U(i - 1, j, k);
            const double uyp = U(i, j + 1, k), uym = U(i, j - 1, k);
            const double uzp = U(i, j, k + 1), uzm = U(i, j, k - 1);
            const double cp = 0.5 * (u0 + uxp), cm = 0.5 * (uxm + u0);
            double n = (cp * cp - cm * cm) * a.idx;
            const double fy0 = 0.5 * (uym + u0) * 0.5 * (Vv(i - 1, j, k) + Vv(i, j, k));
            const double fy1 = 0.5 * (u0 + uyp) * 0.5 * (Vv(i - 1, j + 1, k) + Vv(i, j + 1, k));
            n += (fy1 - fy0) * a.idy;
            const double fz0 = (wlo0 * uzm + whi0 * u0) * 0.5 * (Ww(i - 1, j, k) + Ww(i, j, k));
            const double fz1 = (wlo1 * u0 + whi1 * uzp) * 0.5 * (Ww(i - 1, j, k + 1) + Ww(i, j, k + 1));
            n += (fz1 - fz0) * idz;
            // Laplacian: faces along x (Dirichlet walls), centres along y
            // (mirrored ghost at walls), centres along z
            const double gym = (j == 0 && wy) ? -u0 : uym, gyp = (j == ny - 1 && wy) ? -u0 : uyp;
            const double lap = (uxm - 2.0 * u0 + uxp) * a.idx2 + (gym - 2.0 * u0 + gyp) * a.idy2 +
                               clo * ((k >= 1 ? uzm : 0.0) - u0) + chi * ((k + 1 < nz ? uzp : 0.0) - u0);
            const double adv = a.gamma * n + (a.rho != 0.0 ? a.rho * a.nu[o] : 0.0);
            ru = a.dt * (-adv + a.inv_re * lap);
            nun = n;
        }
        // ---------------- v at y-face j
        double rv = 0.0, nvn = 0.0;
        if (!(wy && j == 0)) {
            const double v0 = Vv(i, j, k), vyp = Vv(i, j + 1, k), vym = Vv(i, j - 1, k);
            const double vxp = Vv(i + 1, j, k), vxm = Vv(i - 1, j, k);
            const double vzp = Vv(i, j, k + 1), vzm = Vv(i, j, k - 1);
            const double cp = 0.5 * (v0 + vyp), cm = 0.5 * (vym + v0);
            double n = (cp * cp - cm * cm) * a.idy;
            const double fx0 = 0.5 * (vxm + v0) * 0.5 * (U(i, j - 1, k) + U(i, j, k));
            const double fx1 = 0.5 * (v0 + vxp) * 0.5 * (U(i + 1, j - 1, k) + U(i + 1, j, k));
            n += (fx1 - fx0) * a.idx;
            const double fz0 = (wlo0 * vzm + whi0 * v0) * 0.5 * (Ww(i, j - 1, k) + Ww(i, j, k));
            const double fz1 = (wlo1 * v0 + whi1 * vzp) * 0.5 * (Ww(i, j - 1, k + 1) + Ww(i, j, k + 1));
            n += (fz1 - fz0) * idz;
            const double gxm = (i == 0 && wx) ? -v0 : vxm, gxp = (i == nx - 1 && wx) ? -v0 : vxp;
            const double lap = (gxm - 2.0 * v0 + gxp) * a.idx2 + (vym - 2.0 * v0 + vyp) * a.idy2 +
                               clo * ((k >= 1 ? vzm : 0.0) - v0) + chi * ((k + 1 < nz ? vzp : 0.0) - v0);
            const double adv = a.gamma * n + (a.rho != 0.0 ? a.rho * a.nv[o] : 0.0);
            rv = a.dt * (-adv + a.inv_re * lap);
            nvn = n;
        }
        // ---------------- w at z-face k
        double rw = 0.0, nwn = 0.0;
        if (k >= 1) {
            const double w0 = Ww(i, j, k), wzp = Ww(i, j, k + 1), wzm = Ww(i, j, k - 1);
            const double wxp = Ww(i + 1, j, k), wxm = Ww(i - 1, j, k);
            const double wyp = Ww(i, j + 1, k), wym = Ww(i, j - 1, k);
            const double cp = 0.5 * (w0 + wzp), cm = 0.5 * (wzm + w0);
            double n = (cp * cp - cm * cm) * ihk;
            // u and v interpolated in z to face k at x-faces i, i+1 / y-faces j, j+1
            const double ui0 = wlo0 * U(i, j, k - 1) + whi0 * U(i, j, k);
            const double ui1 = wlo0 * U(i + 1, j, k - 1) + whi0 * U(i + 1, j, k);
            n += (0.5 * (w0 + wxp) * ui1 - 0.5 * (wxm + w0) * ui0) * a.idx;
            const double vi0 = wlo0 * Vv(i, j, k - 1) + whi0 * Vv(i, j, k);
            const double vi1 = wlo0 * Vv(i, j + 1, k - 1) + whi0 * Vv(i, j + 1, k);
            n += (0.5 * (w0 + wyp) * vi1 - 0.5 * (wym + w0) * vi0) * a.idy;
            const double gxm = (i == 0 && wx) ? -w0 : wxm, gxp = (i == nx - 1 && wx) ? -w0 : wxp;
            const double gym = (j == 0 && wy) ? -w0 : wym, gyp = (j == ny - 1 && wy) ? -w0 : wyp;
            const double lap = (gxm - 2.0 * w0 + gxp) * a.idx2 + (gym - 2.0 * w0 + gyp) * a.idy2 + flo * wzm +
                               fhi * wzp - fdg * w0;
            const double adv = a.gamma * n + (a.rho != 0.0 ? a.rho * a.nw[o] : 0.0);
            rw = a.dt * (-adv + a.inv_re * lap);
            nwn = n;
        }
        a.ru[o] = ru;
        a.rv[o] = rv;
        a.rw[o] = rw;
        a.nu[o] = nun;
        a.nv[o] = nvn;
        a.nw[o] = nwn;
    }
}

// The same right-hand side with one lane per pair of adjacent cells (i0,
// i0 + 1), i0 even: every row the stencils touch is read as one aligned
// 16-byte pair plus its two x neighbours, each (row, column) once per lane.
// Needs nx even and 16-byte aligned fields.  Same tile order as above.
template <int NT, int GJ, bool NTS = false>   // NTS: non-temporal stores of the six outputs
__global__ __launch_bounds__(NT) void k_momentum_rhs_pairs(MomArgs a) {
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int b = (int)xcd_remap(blockIdx.x, gridDim.x);
    const int per = nz * GJ;
    const int jt = b / per;
    const int rem = b - jt * per;
    const int k = rem / GJ;
    const int j = jt * GJ + (rem - k * GJ);
    const size_t nxy = (size_t)nx * ny;
    const bool wx = !a.perx, wy = !a.pery;
    // row pointers (nullptr: outside the grid at a wall, or a dead wall row)
    auto rowp = [&](const double* f, int jj, int kk, bool deadj0, bool deadk0) -> const double* {
        if (kk < 0 || kk >= nz || (deadk0 && kk == 0)) return nullptr;
        if (jj < 0 || jj >= ny) {
            if (wy) return nullptr;
            jj = (jj + ny) % ny;
        }
        if (deadj0 && jj == 0) return nullptr;
        return f + (size_t)kk * nxy + (size_t)jj * nx;
    };
    // values at columns i0-1 .. i0+2 of a row (x walls: 0 outside; periodic:
    // wrapped); dead0: column 0 is a dead wall face (u with x walls)
    auto win = [&](const double* r, int i0, bool dead0, double (&q)[4]) {
        if (!r) {
            q[0] = q[1] = q[2] = q[3] = 0.0;
            return;
        }
        const double2 c = *reinterpret_cast<const double2*>(r + i0);
        q[1] = c.x;
        q[2] = c.y;
        q[0] = (i0 > 0) ? r[i0 - 1] : (wx ? 0.0 : r[nx - 1]);
        q[3] = (i0 + 2 < nx) ? r[i0 + 2] : (wx ? 0.0 : r[0]);
        if (dead0 && wx) {
            if (i0 == 0) q[1] = 0.0;
            if (i0 - 1 == 0) q[0] = 0.0;
        }
    };
    const double dzk = a.dz[k];
    const double wlo0 = (k >= 1) ? dzk / (a.dz[k - 1] + dzk) : 0.0;
    const double whi0 = (k >= 1) ? a.dz[k - 1] / (a.dz[k - 1] + dzk) : 0.0;
    const double wlo1 = (k + 1 < nz) ? a.dz[k + 1] / (dzk + a.dz[k + 1]) : 0.0;
    const double whi1 = (k + 1 < nz) ? dzk / (dzk + a.dz[k + 1]) : 0.0;
    const double idz = a.inv_dz[k];
    const double ihk = (k >= 1) ? a.inv_h[k] : 0.0;
    const double clo = (k >= 1) ? a.za[k] : 2.0 * idz * idz;
    const double chi = (k + 1 < nz) ? a.zc[k] : 2.0 * idz * idz;
    const double flo = (k >= 2) ? a.inv_dz[k - 1] * ihk : 0.0;
    const double fhi = (k + 1 < nz) ? idz * ihk : 0.0;
    const double fdg = (k >= 1) ? (a.inv_dz[k - 1] + idz) * ihk : 0.0;
    const size_t row = (size_t)k * nxy + (size_t)j * nx;
    const double* u_c = rowp(a.u, j, k, false, false);
    const double* u_yp = rowp(a.u, j + 1, k, false, false);
    const double* u_ym = rowp(a.u, j - 1, k, false, false);
    const double* u_zp = rowp(a.u, j, k + 1, false, false);
    const double* u_zm = rowp(a.u, j, k - 1, false, false);
    const double* v_c = rowp(a.v, j, k, wy, false);
    const double* v_yp = rowp(a.v, j + 1, k, wy, false);
    const double* v_ym = rowp(a.v, j - 1, k, wy, false);
    const double* v_zp = rowp(a.v, j, k + 1, wy, false);
    const double* v_zm = rowp(a.v, j, k - 1, wy, false);
    const double* v_ypzm = rowp(a.v, j + 1, k - 1, wy, false);
    const double* w_c = rowp(a.w, j, k, false, true);
    const double* w_zp = rowp(a.w, j, k + 1, false, true);
    const double* w_zm = rowp(a.w, j, k - 1, false, true);
    const double* w_yp = rowp(a.w, j + 1, k, false, true);
    const double* w_ym = rowp(a.w, j - 1, k, false, true);
    const double* w_ymzp = rowp(a.w, j - 1, k + 1, false, true);
    const bool vdead = wy && j == 0, wdead = k == 0;
    for (int i0 = 2 * threadIdx.x; i0 < nx; i0 += 2 * NT) {
        double uc[4], uyp[4], uym[4], uzp[4], uzm[4];
        double vc[4], vyp[4], vym[4], vzp[4], vzm[4], vypzm[4];
        double wc[4], wzp[4], wzm[4], wyp[4], wym[4], wymzp[4];
        win(u_c, i0, true, uc);
        win(u_yp, i0, true, uyp);
        win(u_ym, i0, true, uym);
        win(u_zp, i0, true, uzp);
        win(u_zm, i0, true, uzm);
        win(v_c, i0, false, vc);
        win(v_yp, i0, false, vyp);
        win(v_ym, i0, false, vym);
        win(v_zp, i0, false, vzp);
        win(v_zm, i0, false, vzm);
        win(v_ypzm, i0, false, vypzm);
        win(w_c, i0, false, wc);
        win(w_zp, i0, false, wzp);
        win(w_zm, i0, false, wzm);
        win(w_yp, i0, false, wyp);
        win(w_ym, i0, false, wym);
        win(w_ymzp, i0, false, wymzp);
        double2 pu = make_double2(0.0, 0.0), pv = pu, pw = pu;
        if (a.rho != 0.0) {
            pu = *reinterpret_cast<const double2*>(a.nu + row + i0);
            pv = *reinterpret_cast<const double2*>(a.nv + row + i0);
            pw = *reinterpret_cast<const double2*>(a.nw + row + i0);
        }
        double ru[2], rv[2], rw[2], nu[2], nv[2], nw[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int i = i0 + c;
            const int m = c, x = c + 1, pp = c + 2;   // window slots of i-1, i, i+1
            // u at x-face i
            ru[c] = 0.0;
            nu[c] = 0.0;
            if (!(wx && i == 0)) {
                const double u0 = uc[x];
                const double cp = 0.5 * (u0 + uc[pp]), cm = 0.5 * (uc[m] + u0);
                double n = (cp * cp - cm * cm) * a.idx;
                const double fy0 = 0.5 * (uym[x] + u0) * 0.5 * (vc[m] + vc[x]);
                const double fy1 = 0.5 * (u0 + uyp[x]) * 0.5 * (vyp[m] + vyp[x]);
                n += (fy1 - fy0) * a.idy;
                const double fz0 = (wlo0 * uzm[x] + whi0 * u0) * 0.5 * (wc[m] + wc[x]);
                const double fz1 = (wlo1 * u0 + whi1 * uzp[x]) * 0.5 * (wzp[m] + wzp[x]);
                n += (fz1 - fz0) * idz;
                const double gym = (j == 0 && wy) ? -u0 : uym[x], gyp = (j == ny - 1 && wy) ? -u0 : uyp[x];
                const double lap = (uc[m] - 2.0 * u0 + uc[pp]) * a.idx2 + (gym - 2.0 * u0 + gyp) * a.idy2 +
                                   clo * (uzm[x] - u0) + chi * (uzp[x] - u0);
                const double adv = a.gamma * n + a.rho * (c ? pu.y : pu.x);
                ru[c] = a.dt * (-adv + a.inv_re * lap);
                nu[c] = n;
            }
            // v at y-face j
            rv[c] = 0.0;
            nv[c] = 0.0;
            if (!vdead) {
                const double v0 = vc[x];
                const double cp = 0.5 * (v0 + vyp[x]), cm = 0.5 * (vym[x] + v0);
                double n = (cp * cp - cm * cm) * a.idy;
                const double fx0 = 0.5 * (vc[m] + v0) * 0.5 * (uym[x] + uc[x]);
                const double fx1 = 0.5 * (v0 + vc[pp]) * 0.5 * (uym[pp] + uc[pp]);
                n += (fx1 - fx0) * a.idx;
                const double fz0 = (wlo0 * vzm[x] + whi0 * v0) * 0.5 * (wym[x] + wc[x]);
                const double fz1 = (wlo1 * v0 + whi1 * vzp[x]) * 0.5 * (wymzp[x] + wzp[x]);
                n += (fz1 - fz0) * idz;
                const double gxm = (i == 0 && wx) ? -v0 : vc[m], gxp = (i == nx - 1 && wx) ? -v0 : vc[pp];
                const double lap = (gxm - 2.0 * v0 + gxp) * a.idx2 + (vym[x] - 2.0 * v0 + vyp[x]) * a.idy2 +
                                   clo * (vzm[x] - v0) + chi * (vzp[x] - v0);
                const double adv = a.gamma * n + a.rho * (c ? pv.y : pv.x);
                rv[c] = a.dt * (-adv + a.inv_re * lap);
                nv[c] = n;
            }
            // w at z-face k
            rw[c] = 0.0;
            nw[c] = 0.0;
            if (!wdead) {
                const double w0 = wc[x];
                const double cp = 0.5 * (w0 + wzp[x]), cm = 0.5 * (wzm[x] + w0);
                double n = (cp * cp - cm * cm) * ihk;
                const double ui0 = wlo0 * uzm[x] + whi0 * uc[x];
                const double ui1 = wlo0 * uzm[pp] + whi0 * uc[pp];
                n += (0.5 * (w0 + wc[pp]) * ui1 - 0.5 * (wc[m] + w0) * ui0) * a.idx;
                const double vi0 = wlo0 * vzm[x] + whi0 * vc[x];
                const double vi1 = wlo0 * vypzm[x] + whi0 * vyp[x];
                n += (0.5 * (w0 + wyp[x]) * vi1 - 0.5 * (wym[x] + w0) * vi0) * a.idy;
                const double gxm = (i == 0 && wx) ? -w0 : wc[m], gxp = (i == nx - 1 && wx) ? -w0 : wc[pp];
                const double gym = (j == 0 && wy) ? -w0 : wym[x], gyp = (j == ny - 1 && wy) ? -w0 : wyp[x];
                const double lap = (gxm - 2.0 * w0 + gxp) * a.idx2 + (gym - 2.0 * w0 + gyp) * a.idy2 +
                                   flo * wzm[x] + fhi * wzp[x] - fdg * w0;
                const double adv = a.gamma * n + a.rho * (c ? pw.y : pw.x);
                rw[c] = a.dt * (-adv + a.inv_re * lap);
                nw[c] = n;
            }
        }
        typedef double d2 __attribute__((ext_vector_type(2)));
        auto put = [&](double* q, double x0, double x1) {
            d2 v;
            v.x = x0;
            v.y = x1;
            if constexpr (NTS)
                __builtin_nontemporal_store(v, reinterpret_cast<d2*>(q + row + i0));
            else
                *reinterpret_cast<d2*>(q + row + i0) = v;
        };
        put(a.ru, ru[0], ru[1]);
        put(a.rv, rv[0], rv[1]);
        put(a.rw, rw[0], rw[1]);
        put(a.nu, nu[0], nu[1]);
        put(a.nv, nv[0], nv[1]);
        put(a.nw, nw[0], nw[1]);
    }
}

}  // namespace dev
}  // namespace fsei
