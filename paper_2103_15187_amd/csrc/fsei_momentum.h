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

}  // namespace dev
}  // namespace fsei
