// HIP kernels of the pressure projection for gfx950 (MI355X): the z
// tridiagonal solves, the singular zero mode, the gradient correction and the
// partial-sum reduction.  The transform kernels are in fsei_transforms.h.
//
// Pass structure of one projection (fields are (nz, ny, nx), x fastest):
//   k_xfwd   : per pair of x-rows, the cell divergence of u* (or the
//              transposed gradient for the adjoint, or the FP64 residual in
//              refinement) fused with the forward x transform
//   k_yfwd   : per tile of x-columns of one z-plane, forward y transform
//   k_zsolve : per (kx, ky) mode, the z tridiagonal, partitioned over the
//              threads of a workgroup (no global scratch)
//   k_zero_mode : the singular (0,0) mode by prefix sums
//   k_yinv, k_xinv : inverse transforms (x inverse writes or accumulates p)
//   k_grad   : gradient correction of the three velocity components
#pragma once

#include <hip/hip_runtime.h>

#include "fsei_fft.h"
#include "fsei_plan.h"
#include "fsei_transforms.h"

namespace fsei {
namespace dev {

// ---------------------------------------------------------------------------
// z: one tridiagonal per (kx, ky) mode,
//   a_k x_{k-1} + (b0_k + sigma) x_k + c_k x_{k+1} = scale * f_k,
// sigma = lambda_x + lambda_y.  A workgroup holds TXL modes (adjacent kx, same
// ky: coalesced rows of TXL elements) x P chunks of one z-line each.  Every
// thread keeps its chunk (<= LMAX rows) in registers, eliminates its interior
// rows in one downward sweep to express them through the two chunk-end
// unknowns, the chunk-end unknowns of a line are solved as a
// P x P tridiagonal in LDS, and each thread then back-substitutes its chunk.
// `transposed` solves T^T y = g through T^T = dz T dz^{-1} (scale by 1/dz_k on
// load and by dz_k on store).
// ---------------------------------------------------------------------------
template <typename TS, typename TC>
struct ZArgs {
    int nx, ny, nz, L, P, transposed, nlist;
    TS* data;
    const int* list;      // LIST mode: mode indices qy*nx + qx
    TC scale;             // 1/(nx ny)
    TC sigma_thr;         // dense mode: skip lines with |sigma| < sigma_thr
    const TC* za;
    const TC* zc;
    const TC* zb0;
    const TC* dz;
    const TC* inv_dz;
    const TC* lamx;
    const TC* lamy;
};

template <typename TS, typename TC, int TXL, int L, int NT, bool LIST>
__global__ __launch_bounds__(NT) void k_zsolve(ZArgs<TS, TC> a) {
    constexpr int PMAX = NT / TXL;
    __shared__ TC sh[4][NT];
    __shared__ TC ta[PMAX * L], tc[PMAX * L], tb[PMAX * L], tm[PMAX * L], tsi[PMAX * L], tso[PMAX * L];
    const int nx = a.nx, nz = a.nz, P = a.P;
    const int npad = P * L;
    // per-k coefficients staged in LDS, padded to P*L rows with decoupled
    // identity rows (a = c = 0, b = 1, f = 0); the scheduling barriers in the
    // sweeps keep each row's LDS reads next to their use, so the coefficients
    // are re-read per sweep instead of being held in registers
    // tsi: load scale 1/(nx ny) (times 1/dz_k when transposed);
    // tso: store scale 1 (dz_k when transposed)
    for (int k = threadIdx.x; k < npad; k += NT) {
        const bool in = k < nz;
        ta[k] = in ? a.za[k] : (TC)0;
        tc[k] = in ? a.zc[k] : (TC)0;
        tb[k] = in ? a.zb0[k] : (TC)1;   // diagonal b0_k + sigma * tm_k
        tm[k] = in ? (TC)1 : (TC)0;
        tsi[k] = in ? (a.transposed ? a.scale * a.inv_dz[k] : a.scale) : (TC)0;
        tso[k] = in ? (a.transposed ? a.dz[k] : (TC)1) : (TC)0;
    }
    const int ln = threadIdx.x % TXL;
    const int p = threadIdx.x / TXL;
    const size_t stride = (size_t)nx * a.ny;
    int qx, qy;
    bool active;
    if constexpr (LIST) {
        const int li = blockIdx.x * TXL + ln;
        active = li < a.nlist;
        const int line = active ? a.list[li] : 0;
        qy = line / nx;
        qx = line - qy * nx;
    } else {
        qx = blockIdx.x * TXL + ln;
        qy = blockIdx.y;
        active = qx < nx;
    }
    TC sigma = (TC)-1;
    if (active) {
        sigma = a.lamx[qx] + a.lamy[qy];
        if (qx == 0 && qy == 0) active = false;
        if constexpr (!LIST) {
            if (fabs(sigma) < a.sigma_thr) active = false;
        }
        if (!active) sigma = (TC)-1;
    }
    const bool inrange = p < P;
    const int s0 = inrange ? p * L : 0;
    TS* __restrict__ col = a.data + (size_t)qy * nx + qx;
    const bool ld = active && inrange;

    TC F[L], Rr[L];
#pragma unroll
    for (int t = 0; t < L; ++t) {
        const int k = s0 + t;
        F[t] = (ld && k < nz) ? (TC)col[(size_t)k * stride] : (TC)0;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < L; ++t) F[t] *= tsi[s0 + t];
    // diagonal of row k: b0_k + sigma, 1 on padding rows (branch free)
#define ZDIAG(k) (tb[k] + sigma * tm[k])
    // One downward sweep over the interior rows s0..s0+L-2 (Dirichlet ends):
    // LU pivots r_t (kept), the eliminated right-hand side d' and the
    // sensitivity g to the left end value.  The back substitution of the
    // first interior row, x_s = sum_t d'_t pi_t with pi_t = prod_{j<t} (-c'_j),
    // is accumulated on the way, so no upward sweep is needed.
    TC cp = 0, dp = 0, g = 1, pi = 1, ysum = 0, gsum = 0;
#pragma unroll
    for (int t = 0; t < L - 1; ++t) {
        const int k = s0 + t;
        const TC A = ta[k], C = tc[k], B = ZDIAG(k);
        const TC r = (TC)1 / (B - A * cp);
        Rr[t] = r;
        dp = (F[t] - A * dp) * r;
        g = -A * g * r;
        ysum += dp * pi;
        gsum += g * pi;
        cp = C * r;
        pi *= -cp;
        __builtin_amdgcn_sched_barrier(0);
    }
    const TC Ylast = dp, Glast = g, Hlast = -cp;
    const TC dh = ysum, ch = -gsum, hh = pi;
    const int me = threadIdx.x;
    // publish first-row expressions for the left neighbour chunk
    sh[0][me] = dh;    // Y_first
    sh[1][me] = -ch;   // G_first
    sh[2][me] = hh;    // H_first
    __syncthreads();
    // reduced row p: alpha x_{e(p-1)} + beta x_{e(p)} + gamma x_{e(p+1)} = phi
    TC al = 0, be = 1, ga = 0, ph = 0;
    if (inrange) {
        const int e = s0 + L - 1;
        const TC Ae = ta[e], Ce = tc[e], Be = ZDIAG(e);
        al = Ae * Glast;
        be = Be + Ae * Hlast;
        ph = F[L - 1] - Ae * Ylast;
        if (p + 1 < P) {
            const int nb = me + TXL;
            be += Ce * sh[1][nb];
            ga = Ce * sh[2][nb];
            ph -= Ce * sh[0][nb];
        }
    }
#undef ZDIAG
    // The P x P reduced system of each line is diagonally dominant like the
    // original; solve it by parallel cyclic reduction over the P threads of
    // the line: at stride s every row eliminates its couplings to rows p-s
    // and p+s (rows outside [0, P) act as identity rows), until all rows are
    // decoupled after ceil(log2 P) steps.
    for (int s = 1; s < P; s <<= 1) {
        __syncthreads();
        sh[0][me] = al;
        sh[1][me] = be;
        sh[2][me] = ga;
        sh[3][me] = ph;
        __syncthreads();
        if (inrange) {
            TC k1 = 0, k2 = 0, alm = 0, gam = 0, phm = 0, alp = 0, gap = 0, php = 0;
            if (p - s >= 0) {
                const int id = me - s * TXL;
                k1 = al / sh[1][id];
                alm = sh[0][id];
                gam = sh[2][id];
                phm = sh[3][id];
            }
            if (p + s < P) {
                const int id = me + s * TXL;
                k2 = ga / sh[1][id];
                alp = sh[0][id];
                gap = sh[2][id];
                php = sh[3][id];
            }
            be = be - k1 * gam - k2 * alp;
            ph = ph - k1 * phm - k2 * php;
            al = -k1 * alm;
            ga = -k2 * gap;
        }
    }
    __syncthreads();
    sh[0][me] = ph / be;   // chunk-end value x_{e(p)}
    __syncthreads();
    const TC XR = sh[0][me];
    const TC XL = (p > 0) ? sh[0][me - TXL] : (TC)0;
    // sweep 3 (down) with the true left value, sweep 4 (up) from the right value
    TC prev = XL;
#pragma unroll
    for (int t = 0; t < L - 1; ++t) {
        prev = (F[t] - ta[s0 + t] * prev) * Rr[t];
        F[t] = prev;
        __builtin_amdgcn_sched_barrier(0);
    }
    F[L - 1] = XR;
    TC nxt = XR;
#pragma unroll
    for (int t = L - 2; t >= 0; --t) {
        nxt = F[t] - tc[s0 + t] * Rr[t] * nxt;
        F[t] = nxt;
        __builtin_amdgcn_sched_barrier(0);
    }
    if (ld) {
        // fresh base address (opaque to the compiler) so the per-row load
        // addresses are not kept alive until the stores
        TS* out = col + (size_t)s0 * stride;
        asm volatile("" : "+v"(out));
#pragma unroll
        for (int t = 0; t < L; ++t) {
            if (s0 + t < nz) out[(size_t)t * stride] = (TS)(F[t] * tso[s0 + t]);
        }
    }
}

// ---------------------------------------------------------------------------
// (0,0) mode: singular z line (zero-flux walls).  Removes the dz-weighted
// mean of the scaled right-hand side (compatibility), integrates the flux
// F_k = sum_{k'<k} dz_k' f_k', sums p_k = sum_{k'<=k} h_k' F_k', and pins
// sum dz_k p_k = 0.  One workgroup of 256 threads, FP64 arithmetic.
// ---------------------------------------------------------------------------
template <typename TS>
struct ZeroArgs {
    int nz, transposed;
    size_t stride;
    TS* data;
    double scale, lz;
    const double* dz;
    const double* inv_dz;
    const double* h;
    double* scal;   // scal[0] <- removed mean (not for the transposed solve)
};

__device__ __forceinline__ double zm_block_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int t = 0; t < 256; ++t) s += sh[t];
        sh[256] = s;
    }
    __syncthreads();
    const double r = sh[256];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double zm_block_exscan(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int t = 0; t < 256; ++t) {
            const double x = sh[t];
            sh[t] = s;
            s += x;
        }
    }
    __syncthreads();
    const double r = sh[threadIdx.x];
    __syncthreads();
    return r;
}

template <typename TS>
__global__ __launch_bounds__(256) void k_zero_mode(ZeroArgs<TS> a) {
    __shared__ double sh[257];
    constexpr int CMAX = kMaxNz / 256;
    const int nz = a.nz;
    const int c = (nz + 255) / 256;
    const int k0 = threadIdx.x * c;
    double f[CMAX];
#pragma unroll
    for (int r = 0; r < CMAX; ++r) {
        const int k = k0 + r;
        f[r] = 0.0;
        if (r < c && k < nz) {
            double sc = a.scale;
            if (a.transposed) sc *= a.inv_dz[k];
            f[r] = (double)a.data[(size_t)k * a.stride] * sc;
        }
    }
    double loc = 0.0;
#pragma unroll
    for (int r = 0; r < CMAX; ++r)
        if (r < c && k0 + r < nz) loc += a.dz[k0 + r] * f[r];
    const double mean = zm_block_sum(loc, sh) / a.lz;
    loc = 0.0;
#pragma unroll
    for (int r = 0; r < CMAX; ++r)
        if (r < c && k0 + r < nz) {
            f[r] -= mean;
            loc += a.dz[k0 + r] * f[r];
        }
    double run = zm_block_exscan(loc, sh);   // flux entering this thread's first row
    double hf[CMAX];
    loc = 0.0;
#pragma unroll
    for (int r = 0; r < CMAX; ++r) {
        hf[r] = 0.0;
        if (r < c && k0 + r < nz) {
            const int k = k0 + r;
            hf[r] = a.h[k] * run;   // h_0 = 0
            run += a.dz[k] * f[r];
            loc += hf[r];
        }
    }
    run = zm_block_exscan(loc, sh);
    loc = 0.0;
#pragma unroll
    for (int r = 0; r < CMAX; ++r) {
        if (r < c && k0 + r < nz) {
            run += hf[r];
            f[r] = run;
            loc += a.dz[k0 + r] * f[r];
        }
    }
    const double pm = zm_block_sum(loc, sh) / a.lz;
#pragma unroll
    for (int r = 0; r < CMAX; ++r) {
        const int k = k0 + r;
        if (r < c && k < nz) {
            double v = f[r] - pm;
            if (a.transposed) v *= a.dz[k];
            a.data[(size_t)k * a.stride] = (TS)v;
        }
    }
    if (threadIdx.x == 0 && !a.transposed && a.scal) a.scal[0] = mean;
}

// ---------------------------------------------------------------------------
// gradient correction on the faces:
//   u += cx (p_i - p_{i-1}),  v += cy (p_j - p_{j-1}),
//   w += sw (bk_k p_k - gk_k p_{k-1});  wall faces written 0.
// forward: cx = -dt/dx, cy = -dt/dy, sw = -dt, bk = gk = 1/h_k
// adjoint (u* <- u - D^T s): cx = 1/dx, cy = 1/dy, sw = 1, bk = 1/dz_k,
//   gk = 1/dz_{k-1}
// ---------------------------------------------------------------------------
template <typename TIO, typename TP>
struct GradArgs {
    int nx, ny, nz, bcx, bcy;
    TIO* u;
    TIO* v;
    TIO* w;
    const TP* p;
    TIO cx, cy, sw;
    const TIO* bk;
    const TIO* gk;
};

template <typename TIO, typename TP>
__global__ __launch_bounds__(256) void k_grad(GradArgs<TIO, TP> a) {
    // one x-row (k, j) per workgroup, rows in XCD-contiguous order so the
    // j-1 and k-1 neighbour rows of p are mostly L2 hits
    const long row = xcd_remap(blockIdx.x, gridDim.x);
    const int nx = a.nx, ny = a.ny;
    const int k = (int)(row / ny);
    const int j = (int)(row - (long)k * ny);
    const size_t base = (size_t)row * nx;
    TIO* __restrict__ u = a.u;
    TIO* __restrict__ v = a.v;
    TIO* __restrict__ w = a.w;
    const TP* __restrict__ p = a.p;
    const TIO bk = a.bk[k], gk = a.gk[k];
    const size_t jm = (j > 0) ? (size_t)nx : (size_t)0 - (size_t)(ny - 1) * nx;   // offset to row j-1
#pragma unroll 4
    for (int i = threadIdx.x; i < nx; i += 256) {
        const size_t idx = base + i;
        const TIO pc = (TIO)p[idx];
        const TIO px = (TIO)p[(i > 0) ? idx - 1 : idx + nx - 1];
        const TIO py = (TIO)p[idx - jm];
        const TIO pz = (k > 0) ? (TIO)p[idx - (size_t)nx * ny] : (TIO)0;
        const TIO uo = u[idx], vo = v[idx], wo = w[idx];
        u[idx] = (a.bcx == FSEI_BC_WALL && i == 0) ? (TIO)0 : uo + a.cx * (pc - px);
        v[idx] = (a.bcy == FSEI_BC_WALL && j == 0) ? (TIO)0 : vo + a.cy * (pc - py);
        w[idx] = (k == 0) ? (TIO)0 : wo + a.sw * (bk * pc - gk * pz);
    }
}

// deterministic sum of the per-block partials (one workgroup)
__global__ __launch_bounds__(256) void k_sum_partials(const double* part, int nblk, double* out) {
    __shared__ double sh[2 * 4];
    double a = 0.0, b = 0.0;
    for (int t = threadIdx.x; t < nblk; t += 256) {
        a += part[2 * t];
        b += part[2 * t + 1];
    }
    block_sum2<256>(a, b, sh);
    if (threadIdx.x == 0) {
        out[0] = a;
        out[1] = b;
    }
}

}  // namespace dev
}  // namespace fsei
