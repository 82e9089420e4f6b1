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
// Reciprocal for the tridiagonal sweeps: the hardware estimate refined by
// Newton steps r <- r + r (1 - x r) (two in FP64, one in FP32), within a
// few ulp of 1/x for the well-scaled pivots of these systems (|x| between
// the smallest z coefficient and |lambda_x + lambda_y|).  The IEEE-exact
// division the compiler emits otherwise is a chain of ten dependent
// instructions on the critical path of every row.
__device__ __forceinline__ double zrcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float zrcp(float x) {
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

template <typename TS, typename TC>
struct ZArgs {
    int nx, ny, nz, L, P, transposed;
    TS* data;
    TC scale;             // 1/(nx ny)
    // skip the lines with |lamx64 + lamy64| < sigma_thr, tested in FP64 on
    // the FP64 tables with the host's own expression, so that a line is
    // solved here exactly when the host left it out of its near-singular list
    double sigma_thr;
    const double* lamx64;
    const double* lamy64;
    const TC* za;
    const TC* zc;
    const TC* zb0;
    const TC* dz;
    const TC* inv_dz;
    const TC* lamx;
    const TC* lamy;
};

template <typename TS, typename TC, int TXL, int L, int NT>
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
    const int qx = blockIdx.x * TXL + ln;
    const int qy = blockIdx.y;
    bool active = qx < nx;
    TC sigma = (TC)-1;
    if (active) {
        sigma = a.lamx[qx] + a.lamy[qy];
        if (qx == 0 && qy == 0) active = false;
        if (fabs(a.lamx64[qx] + a.lamy64[qy]) < a.sigma_thr) active = false;
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
        const TC r = zrcp(B - A * cp);
        Rr[t] = r;
        dp = (F[t] - A * dp) * r;
        g = -A * g * r;
        ysum += dp * pi;
        gsum += g * pi;
        cp = C * r;
        pi *= -cp;
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
                k1 = al * zrcp(sh[1][id]);
                alm = sh[0][id];
                gam = sh[2][id];
                phm = sh[3][id];
            }
            if (p + s < P) {
                const int id = me + s * TXL;
                k2 = ga * zrcp(sh[1][id]);
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
    sh[0][me] = ph * zrcp(be);   // chunk-end value x_{e(p)}
    __syncthreads();
    const TC XR = sh[0][me];
    const TC XL = (p > 0) ? sh[0][me - TXL] : (TC)0;
    // sweep 3 (down) with the true left value, sweep 4 (up) from the right value
    TC prev = XL;
#pragma unroll
    for (int t = 0; t < L - 1; ++t) {
        prev = (F[t] - ta[s0 + t] * prev) * Rr[t];
        F[t] = prev;
    }
    F[L - 1] = XR;
    TC nxt = XR;
#pragma unroll
    for (int t = L - 2; t >= 0; --t) {
        nxt = F[t] - tc[s0 + t] * Rr[t] * nxt;
        F[t] = nxt;
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
// Same solver with M adjacent modes (qx .. qx+M-1) per lane: the global
// accesses become one M-wide vector (16 bytes for two FP64 or four FP32
// modes) and a workgroup row segment covers M*TXLM modes (256 B), which
// streams markedly better from HBM than 128-B segments; the M lines'
// recurrences also interleave.  Dense mode only; needs nx % M == 0.
// ---------------------------------------------------------------------------
// M adjacent values as one native vector (one 8- or 16-byte access)
template <typename T, int M> struct VecM;
template <> struct VecM<double, 2> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct VecM<float, 2> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct VecM<float, 4> { typedef float type __attribute__((ext_vector_type(4))); };

template <typename TS, typename TC, int M, int TXLM, int L, int NT>
__global__ __launch_bounds__(NT) void k_zsolvev(ZArgs<TS, TC> a) {
    using V = typename VecM<TS, M>::type;
    constexpr int PMAX = NT / TXLM;
    __shared__ TC sh[4][M * NT];
    __shared__ TC ta[PMAX * L], tc[PMAX * L], tb[PMAX * L], tm[PMAX * L], tsi[PMAX * L], tso[PMAX * L];
    const int nx = a.nx, nz = a.nz, P = a.P;
    const int npad = P * L;
    for (int k = threadIdx.x; k < npad; k += NT) {
        const bool in = k < nz;
        ta[k] = in ? a.za[k] : (TC)0;
        tc[k] = in ? a.zc[k] : (TC)0;
        tb[k] = in ? a.zb0[k] : (TC)1;   // diagonal b0_k + sigma * tm_k
        tm[k] = in ? (TC)1 : (TC)0;
        tsi[k] = in ? (a.transposed ? a.scale * a.inv_dz[k] : (TC)1) : (TC)0;
        tso[k] = in ? (a.transposed ? a.dz[k] : a.scale) : (TC)0;
    }
    const int ln = threadIdx.x % TXLM;
    const int p = threadIdx.x / TXLM;
    const int qx0 = (blockIdx.x * TXLM + ln) * M;
    const int qy = blockIdx.y;
    const size_t strideV = (size_t)nx * a.ny / M;   // in vectors
    bool act[M];
    TC sigma[M];
    bool anyl = false, alll = true;
#pragma unroll
    for (int h = 0; h < M; ++h) {
        const int qx = qx0 + h;
        act[h] = qx < nx;
        sigma[h] = (TC)-1;
        if (act[h]) {
            sigma[h] = a.lamx[qx] + a.lamy[qy];
            if ((qx == 0 && qy == 0) || fabs(a.lamx64[qx] + a.lamy64[qy]) < a.sigma_thr) act[h] = false;
            if (!act[h]) sigma[h] = (TC)-1;
        }
        anyl = anyl || act[h];
        alll = alll && act[h];
    }
    const bool inrange = p < P;
    const int s0 = inrange ? p * L : 0;
    const bool anyact = anyl && inrange;
    const size_t coff = (size_t)qy * nx + (qx0 < nx ? qx0 : 0);   // element offset of the lane's column
    const V* __restrict__ col = reinterpret_cast<const V*>(a.data + coff);

    TC F[M][L], Rr[M][L];
#pragma unroll
    for (int t = 0; t < L; ++t) {
        const int k = s0 + t;
        V v = (V)(TS)0;
        if (anyact && k < nz) v = col[(size_t)k * strideV];
#pragma unroll
        for (int h = 0; h < M; ++h) F[h][t] = (TC)v[h];
    }
    __syncthreads();
    // the forward solve's uniform 1/(nx ny) is applied at the store (one
    // multiply fewer per value); the transposed solve's 1/dz_k here
    if (a.transposed) {
#pragma unroll
        for (int t = 0; t < L; ++t)
#pragma unroll
            for (int h = 0; h < M; ++h) F[h][t] *= tsi[s0 + t];
    }
    // downward sweep of the M lines (interleaved), first-row back
    // substitution accumulated as running sums (see k_zsolve)
    TC cp[M], dp[M], g[M], pi[M], ys[M], gs[M];
#pragma unroll
    for (int h = 0; h < M; ++h) {
        cp[h] = 0;
        dp[h] = 0;
        g[h] = 1;
        pi[h] = 1;
        ys[h] = 0;
        gs[h] = 0;
    }
#pragma unroll
    for (int t = 0; t < L - 1; ++t) {
        const int k = s0 + t;
        const TC A = ta[k], C = tc[k], B0 = tb[k], Mk = tm[k];
#pragma unroll
        for (int h = 0; h < M; ++h) {
            const TC r = zrcp(B0 + sigma[h] * Mk - A * cp[h]);
            Rr[h][t] = r;
            dp[h] = (F[h][t] - A * dp[h]) * r;
            g[h] = -A * g[h] * r;
            ys[h] += dp[h] * pi[h];
            gs[h] += g[h] * pi[h];
            cp[h] = C * r;
            pi[h] *= -cp[h];
        }
    }
    const int me = threadIdx.x;
    TC al[M], be[M], ga[M], ph[M];
#pragma unroll
    for (int h = 0; h < M; ++h) {
        sh[0][M * me + h] = ys[h];    // Y_first
        sh[1][M * me + h] = gs[h];    // G_first
        sh[2][M * me + h] = pi[h];    // H_first
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < M; ++h) {
        al[h] = 0;
        be[h] = 1;
        ga[h] = 0;
        ph[h] = 0;
        if (inrange) {
            const int e = s0 + L - 1;
            const TC Ae = ta[e], Ce = tc[e], Be = tb[e] + sigma[h] * tm[e];
            al[h] = Ae * g[h];
            be[h] = Be - Ae * cp[h];
            ph[h] = F[h][L - 1] - Ae * dp[h];
            if (p + 1 < P) {
                const int nb = M * (me + TXLM) + h;
                be[h] += Ce * sh[1][nb];
                ga[h] = Ce * sh[2][nb];
                ph[h] -= Ce * sh[0][nb];
            }
        }
    }
    // parallel cyclic reduction of the reduced systems of the M lines
    for (int s = 1; s < P; s <<= 1) {
        __syncthreads();
#pragma unroll
        for (int h = 0; h < M; ++h) {
            sh[0][M * me + h] = al[h];
            sh[1][M * me + h] = be[h];
            sh[2][M * me + h] = ga[h];
            sh[3][M * me + h] = ph[h];
        }
        __syncthreads();
        if (inrange) {
#pragma unroll
            for (int h = 0; h < M; ++h) {
                TC k1 = 0, k2 = 0, alm = 0, gam = 0, phm = 0, alp = 0, gap = 0, php = 0;
                if (p - s >= 0) {
                    const int id = M * (me - s * TXLM) + h;
                    k1 = al[h] * zrcp(sh[1][id]);
                    alm = sh[0][id];
                    gam = sh[2][id];
                    phm = sh[3][id];
                }
                if (p + s < P) {
                    const int id = M * (me + s * TXLM) + h;
                    k2 = ga[h] * zrcp(sh[1][id]);
                    alp = sh[0][id];
                    gap = sh[2][id];
                    php = sh[3][id];
                }
                be[h] = be[h] - k1 * gam - k2 * alp;
                ph[h] = ph[h] - k1 * phm - k2 * php;
                al[h] = -k1 * alm;
                ga[h] = -k2 * gap;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < M; ++h) sh[0][M * me + h] = ph[h] * zrcp(be[h]);
    __syncthreads();
    TC XR[M], prev[M];
#pragma unroll
    for (int h = 0; h < M; ++h) {
        XR[h] = sh[0][M * me + h];
        prev[h] = (p > 0) ? sh[0][M * (me - TXLM) + h] : (TC)0;   // x left of the chunk
    }
#pragma unroll
    for (int t = 0; t < L - 1; ++t) {
        const TC A = ta[s0 + t];
#pragma unroll
        for (int h = 0; h < M; ++h) {
            prev[h] = (F[h][t] - A * prev[h]) * Rr[h][t];
            F[h][t] = prev[h];
        }
    }
#pragma unroll
    for (int h = 0; h < M; ++h) F[h][L - 1] = XR[h];
#pragma unroll
    for (int t = L - 2; t >= 0; --t) {
        const TC C = tc[s0 + t];
#pragma unroll
        for (int h = 0; h < M; ++h) {
            XR[h] = F[h][t] - C * Rr[h][t] * XR[h];
            F[h][t] = XR[h];
        }
    }
    if (anyact) {
        // store addresses rebuilt from the field base (not kept live from the
        // loads), as whole-vector global stores
        size_t ooff = coff + (size_t)s0 * strideV * M;
        asm volatile("" : "+v"(ooff));
        V* out = reinterpret_cast<V*>(a.data + ooff);
        TS* outs = a.data + ooff;
#pragma unroll
        for (int t = 0; t < L; ++t) {
            if (s0 + t < nz) {
                const TC so = tso[s0 + t];
                if (alll) {
                    V v;
#pragma unroll
                    for (int h = 0; h < M; ++h) v[h] = (TS)(F[h][t] * so);
                    out[(size_t)t * strideV] = v;
                } else {
#pragma unroll
                    for (int h = 0; h < M; ++h)
                        if (act[h]) outs[(size_t)t * M * strideV + h] = (TS)(F[h][t] * so);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Persistent form of k_zsolvev for the forward solve on whole tiles (P =
// NT / TXLM chunks of L rows, nz = P L, nx a multiple of M TXLM, 16-byte
// vectors), one workgroup per CU: a workgroup walks tiles b, b + gridDim.x,
// ...; while it solves one tile, the first S rows of every chunk of its next
// tile come into LDS by direct global-to-LDS loads (no registers held), so
// the load phase of a tile covers only its last L - S rows and the rest of
// the tile's bytes arrive while the CU computes.  Each wave reads back only
// the LDS slots its own loads wrote (slot = wave base + lane), so the buffer
// needs no barrier, only the wave's own counters.  Same arithmetic, in the
// same order, as k_zsolvev.
// ---------------------------------------------------------------------------
template <typename TS, typename TC, int M, int TXLM, int L, int NT, int S>
__global__ __launch_bounds__(NT) void k_zsolvev_pf(ZArgs<TS, TC> a) {
    using V = typename VecM<TS, M>::type;
    static_assert(sizeof(V) == 16, "16-byte direct loads");
    static_assert(S >= 1 && S < L, "prefetched rows");
    constexpr int P = NT / TXLM;
    constexpr int NZ = P * L;
    typedef __attribute__((address_space(3))) void* lds_void;
    typedef const __attribute__((address_space(1))) void* glb_void;
    __shared__ TC sh[4][M * NT];
    __shared__ TC ta[NZ], tc[NZ], tb[NZ], tso[NZ];
    __shared__ V pf[S][NT];
    const int nx = a.nx;
    for (int k = threadIdx.x; k < NZ; k += NT) {
        ta[k] = a.za[k];
        tc[k] = a.zc[k];
        tb[k] = a.zb0[k];
        tso[k] = a.scale;   // forward solve only: the uniform 1/(nx ny), applied at the store
    }
    const int ln = threadIdx.x % TXLM;
    const int p = threadIdx.x / TXLM;
    const int s0 = p * L;
    const int wbase = threadIdx.x & ~63;
    const int ntx = nx / (M * TXLM);
    const int ntiles = ntx * a.ny;
    const size_t strideV = (size_t)nx * a.ny / M;   // in vectors
    auto coff = [&](int b) -> size_t {              // element offset of the lane's column in tile b
        const int qy = b / ntx;
        return (size_t)qy * nx + (size_t)((b - qy * ntx) * TXLM + ln) * M;
    };
    auto prefetch = [&](int b) {
        const V* src = reinterpret_cast<const V*>(a.data + coff(b)) + (size_t)s0 * strideV;
#pragma unroll
        for (int t = 0; t < S; ++t)
            __builtin_amdgcn_global_load_lds((glb_void)(src + (size_t)t * strideV), (lds_void)&pf[t][wbase], 16, 0, 0);
    };
    prefetch(blockIdx.x);   // the host launches at most ntiles workgroups
    __syncthreads();
    for (int b = blockIdx.x; b < ntiles; b += gridDim.x) {
        const int qy = b / ntx;
        const int qx0 = (b - qy * ntx) * TXLM * M + ln * M;
        bool act[M];
        TC sigma[M];
        bool anyl = false, alll = true;
#pragma unroll
        for (int h = 0; h < M; ++h) {
            const int qx = qx0 + h;
            const double s64 = a.lamx64[qx] + a.lamy64[qy];
            const TC sg = a.lamx[qx] + a.lamy[qy];
            const bool off = ((qx | qy) == 0) | (fabs(s64) < a.sigma_thr);
            act[h] = !off;
            sigma[h] = off ? (TC)-1 : sg;
            anyl = anyl | act[h];
            alll = alll & act[h];
        }
        // the row stride re-read opaquely each tile, so the compiler rebuilds
        // the row addresses per tile instead of keeping 24 of them live
        size_t sv = strideV;
        asm volatile("" : "+s"(sv));
        const size_t cof = coff(b);
        const V* __restrict__ col = reinterpret_cast<const V*>(a.data + cof) + (size_t)s0 * sv;
        TC F[M][L], Rr[M][L];
#pragma unroll
        for (int t = S; t < L; ++t) {
            const V v = col[(size_t)t * sv];
#pragma unroll
            for (int h = 0; h < M; ++h) F[h][t] = (TC)v[h];
        }
        // rows 0 .. S-1 from this wave's slots (its direct loads for this
        // tile were issued before every load above)
        __builtin_amdgcn_s_waitcnt(imm_wait_vm(L - S));
#pragma unroll
        for (int t = 0; t < S; ++t) {
            const V v = pf[t][threadIdx.x];
#pragma unroll
            for (int h = 0; h < M; ++h) F[h][t] = (TC)v[h];
        }
        __builtin_amdgcn_s_waitcnt(imm_wait_lgkm0());   // buffer read: free for the next tile's rows
        TC cp[M], dp[M], g[M], pi[M], ys[M], gs[M];
#pragma unroll
        for (int h = 0; h < M; ++h) {
            cp[h] = 0;
            dp[h] = 0;
            g[h] = 1;
            pi[h] = 1;
            ys[h] = 0;
            gs[h] = 0;
        }
#pragma unroll
        for (int t = 0; t < L - 1; ++t) {
            const int k = s0 + t;
            const TC A = ta[k], C = tc[k], B0 = tb[k];
#pragma unroll
            for (int h = 0; h < M; ++h) {
                const TC r = zrcp(B0 + sigma[h] - A * cp[h]);
                Rr[h][t] = r;
                dp[h] = (F[h][t] - A * dp[h]) * r;
                g[h] = -A * g[h] * r;
                ys[h] += dp[h] * pi[h];
                gs[h] += g[h] * pi[h];
                cp[h] = C * r;
                pi[h] *= -cp[h];
            }
        }
        // the next tile's first rows: issued once the downward sweep has used
        // every register row (a wait for a register row behind them would
        // wait for them too), in flight through the reduction and the sweeps
        __builtin_amdgcn_sched_barrier(0);
        {
            const int nb = b + (int)gridDim.x;
            prefetch(nb < ntiles ? nb : b);   // the last tile re-reads its own rows (never used)
        }
        __builtin_amdgcn_sched_barrier(0);
        const int me = threadIdx.x;
        TC al[M], be[M], ga[M], ph[M];
#pragma unroll
        for (int h = 0; h < M; ++h) {
            sh[0][M * me + h] = ys[h];
            sh[1][M * me + h] = gs[h];
            sh[2][M * me + h] = pi[h];
        }
        sync_lds_nofence();
#pragma unroll
        for (int h = 0; h < M; ++h) {
            const int e = s0 + L - 1;
            const TC Ae = ta[e], Ce = tc[e], Be = tb[e] + sigma[h];
            al[h] = Ae * g[h];
            be[h] = Be - Ae * cp[h];
            ph[h] = F[h][L - 1] - Ae * dp[h];
            ga[h] = 0;
            if (p + 1 < P) {
                const int nb = M * (me + TXLM) + h;
                be[h] += Ce * sh[1][nb];
                ga[h] = Ce * sh[2][nb];
                ph[h] -= Ce * sh[0][nb];
            }
        }
        for (int s = 1; s < P; s <<= 1) {
            sync_lds_nofence();
#pragma unroll
            for (int h = 0; h < M; ++h) {
                sh[0][M * me + h] = al[h];
                sh[1][M * me + h] = be[h];
                sh[2][M * me + h] = ga[h];
                sh[3][M * me + h] = ph[h];
            }
            sync_lds_nofence();
#pragma unroll
            for (int h = 0; h < M; ++h) {
                TC k1 = 0, k2 = 0, alm = 0, gam = 0, phm = 0, alp = 0, gap = 0, php = 0;
                if (p - s >= 0) {
                    const int id = M * (me - s * TXLM) + h;
                    k1 = al[h] * zrcp(sh[1][id]);
                    alm = sh[0][id];
                    gam = sh[2][id];
                    phm = sh[3][id];
                }
                if (p + s < P) {
                    const int id = M * (me + s * TXLM) + h;
                    k2 = ga[h] * zrcp(sh[1][id]);
                    alp = sh[0][id];
                    gap = sh[2][id];
                    php = sh[3][id];
                }
                be[h] = be[h] - k1 * gam - k2 * alp;
                ph[h] = ph[h] - k1 * phm - k2 * php;
                al[h] = -k1 * alm;
                ga[h] = -k2 * gap;
            }
        }
        sync_lds_nofence();
#pragma unroll
        for (int h = 0; h < M; ++h) sh[0][M * me + h] = ph[h] * zrcp(be[h]);
        sync_lds_nofence();
        TC XR[M], prev[M];
#pragma unroll
        for (int h = 0; h < M; ++h) {
            XR[h] = sh[0][M * me + h];
            prev[h] = (p > 0) ? sh[0][M * (me - TXLM) + h] : (TC)0;
        }
#pragma unroll
        for (int t = 0; t < L - 1; ++t) {
            const TC A = ta[s0 + t];
#pragma unroll
            for (int h = 0; h < M; ++h) {
                prev[h] = (F[h][t] - A * prev[h]) * Rr[h][t];
                F[h][t] = prev[h];
            }
        }
#pragma unroll
        for (int h = 0; h < M; ++h) F[h][L - 1] = XR[h];
#pragma unroll
        for (int t = L - 2; t >= 0; --t) {
            const TC C = tc[s0 + t];
#pragma unroll
            for (int h = 0; h < M; ++h) {
                XR[h] = F[h][t] - C * Rr[h][t] * XR[h];
                F[h][t] = XR[h];
            }
        }
        if (anyl) {
            size_t ooff = cof + (size_t)s0 * strideV * M;
            asm volatile("" : "+v"(ooff));
            V* out = reinterpret_cast<V*>(a.data + ooff);
            TS* outs = a.data + ooff;
#pragma unroll
            for (int t = 0; t < L; ++t) {
                const TC so = tso[s0 + t];
                if (alll) {
                    V v;
#pragma unroll
                    for (int h = 0; h < M; ++h) v[h] = (TS)(F[h][t] * so);
                    out[(size_t)t * strideV] = v;
                } else {
#pragma unroll
                    for (int h = 0; h < M; ++h)
                        if (act[h]) outs[(size_t)t * M * strideV + h] = (TS)(F[h][t] * so);
                }
            }
        }
        sync_lds_nofence();   // sh is rewritten by the next tile
    }
    __builtin_amdgcn_s_waitcnt(0);   // the last direct loads land before the workgroup's LDS is released
}

// ---------------------------------------------------------------------------
// Near-singular mode lines: |lambda_x + lambda_y| below the plan's threshold
// (condition 1 + 4 / (dz_min^2 |sigma|) above 1e4).  One lane per line,
// sequential Thomas in FP64 with the pivots in row-sum form.  With zero-flux
// walls every row of L_z + sigma sums to sigma, so the pivot
//     d_k = b_k - a_k c_{k-1} / d_{k-1},   b_k = -(a_k + c_k) + sigma,
// equals g_k - c_k with g_k = sigma - a_k g_{k-1} / d_{k-1}, g_0 = sigma: every
// term has the sign of sigma, nothing cancels.  Forming b_k first rounds the
// small sigma against a_k + c_k, which costs up to ~1e-11 relative error at
// condition 1e8 in FP64 (768 x 768 x 1024, tanh 3.0); this form stays at
// ~1e-15.  The eliminated right-hand side and the ratios c_k / d_k go to an
// FP64 scratch (line-contiguous across lanes: coalesced), the back
// substitution writes the field.
// ---------------------------------------------------------------------------
template <typename TS>
struct ZSeqArgs {
    int nx, nz, nlist, transposed;
    size_t stride;          // nx * ny
    TS* data;
    const int* list;        // line indices qy * nx + qx, ascending
    double* ys;             // scratch, nlist * nz: eliminated right-hand side
    double* cps;            // scratch, nlist * nz: c_k / d_k
    const double* za;
    const double* zc;
    const double* lamx;
    const double* lamy;
    const double* dz;       // transposed solve: input scaled by 1/dz_k, output by dz_k
    double scale;           // 1 / (nx ny)
};

template <typename TS>
__global__ __launch_bounds__(64) void k_zline_seq(ZSeqArgs<TS> a) {
    // The per-row coefficients go to LDS first (uniform reads there, off the
    // critical path of the recurrences).  Rows go in batches of B with the
    // next batch's loads issued before the current batch is eliminated; the
    // batch bodies have no branches (row indices of loads are clamped into
    // the line, and the last nz % B rows are a separate tail), so the
    // compiler waits only for the batch it uses.
    constexpr int B = 16;
    __shared__ double sa[kMaxNz], sc[kMaxNz], si[kMaxNz], so[kMaxNz];
    const int nz = a.nz, nl = a.nlist;
    for (int k = threadIdx.x; k < nz; k += 64) {
        sa[k] = (k > 0) ? a.za[k] : 0.0;
        sc[k] = (k + 1 < nz) ? a.zc[k] : 0.0;
        si[k] = a.transposed ? a.scale / a.dz[k] : a.scale;
        so[k] = a.transposed ? a.dz[k] : 1.0;
    }
    __syncthreads();
    const int li = blockIdx.x * 64 + threadIdx.x;
    if (li >= nl) return;
    const int line = a.list[li];
    const int qy = line / a.nx, qx = line - qy * a.nx;
    const double sigma = a.lamx[qx] + a.lamy[qy];
    const TS* __restrict__ colr = a.data + line;
    TS* __restrict__ colw = a.data + line;
    const size_t st = a.stride;
    double* __restrict__ ys = a.ys + li;
    double* __restrict__ cps = a.cps + li;
    const int nfull = nz - nz % B;
    auto load_rows = [&](int k0, double* f) {
#pragma unroll
        for (int t = 0; t < B; ++t) {
            const int k = (k0 + t < nz) ? k0 + t : nz - 1;   // clamped (the value is then unused)
            f[t] = (double)colr[(size_t)k * st];
        }
    };
    double q = 1.0, y = 0.0;   // q = g_{k-1} / d_{k-1} (1 before the first row)
    auto fwd_row = [&](int k, double f) {
        const double A = sa[k], C = sc[k];
        const double g = sigma - A * q;
        const double r = zrcp(g - C);
        q = g * r;
        y = (f * si[k] - A * y) * r;
        ys[(size_t)k * nl] = y;
        cps[(size_t)k * nl] = C * r;
    };
    double fa[B], fb[B];
    load_rows(0, fa);
    for (int k0 = 0; k0 < nfull; k0 += B) {
        load_rows(k0 + B, fb);
#pragma unroll
        for (int t = 0; t < B; ++t) fwd_row(k0 + t, fa[t]);
#pragma unroll
        for (int t = 0; t < B; ++t) fa[t] = fb[t];
    }
#pragma unroll
    for (int t = 0; t < B; ++t)
        if (nfull + t < nz) fwd_row(nfull + t, fa[t]);
    // back substitution, top row first: the tail, then the full batches
    auto load_back = [&](int k1, double* yv, double* cv) {   // rows k1, k1 - 1, ..., k1 - B + 1
#pragma unroll
        for (int t = 0; t < B; ++t) {
            const int k = (k1 - t >= 0) ? k1 - t : 0;
            yv[t] = ys[(size_t)k * nl];
            cv[t] = cps[(size_t)k * nl];
        }
    };
    double x = 0.0;
    auto back_row = [&](int k, double yk, double ck) {
        x = yk - ck * x;
        colw[(size_t)k * st] = (TS)(x * so[k]);
    };
    double ya[B], ca[B], yb[B], cb[B];
    load_back(nz - 1, ya, ca);
    if (nfull > 0) load_back(nfull - 1, yb, cb);
    const int rem = nz - nfull;
#pragma unroll
    for (int t = 0; t < B; ++t)
        if (t < rem) back_row(nz - 1 - t, ya[t], ca[t]);
    for (int k1 = nfull - 1; k1 >= 0; k1 -= B) {
#pragma unroll
        for (int t = 0; t < B; ++t) {
            ya[t] = yb[t];
            ca[t] = cb[t];
        }
        load_back(k1 - B, yb, cb);
#pragma unroll
        for (int t = 0; t < B; ++t) back_row(k1 - t, ya[t], ca[t]);
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
    // one x-row (k, j) per workgroup in XCD-contiguous order.  When ny is a
    // multiple of GJ the rows go in tiles of GJ rows, plane by plane inside a
    // tile: the k-1 row of p was read GJ workgroups earlier and the j-1 row
    // one workgroup earlier on the same XCD (L2 hits), except at tile edges
    constexpr int GJ = 8;
    const int b = (int)xcd_remap(blockIdx.x, gridDim.x);
    const int nx = a.nx, ny = a.ny;
    int k, j;
    if (ny % GJ == 0) {
        const int per = a.nz * GJ;
        const int jt = b / per;
        const int rem = b - jt * per;
        k = rem / GJ;
        j = jt * GJ + (rem - k * GJ);
    } else {
        k = b / ny;
        j = b - k * ny;
    }
    const long row = (long)k * ny + j;
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

// One x-row per workgroup, one cell pair per lane (NT >= nx / 2): the
// simplest streaming shape, which runs closest to the HBM ceiling.  Rows in
// tiles of GJ rows (ny % GJ == 0), plane by plane inside a tile (as k_grad).
template <typename TIO, typename TP, int NT, int GJ>
__global__ __launch_bounds__(NT) void k_grad_row2(GradArgs<TIO, TP> a) {
    using V = typename Vec2T<TIO>::type;
    using VP = typename Vec2T<TP>::type;
    const int b = (int)xcd_remap(blockIdx.x, gridDim.x);
    const int nx = a.nx, ny = a.ny;
    const int per = a.nz * GJ;
    const int jt = b / per;
    const int rem = b - jt * per;
    const int k = rem / GJ;
    const int j = jt * GJ + (rem - k * GJ);
    const unsigned i = 2u * threadIdx.x;
    if (i >= (unsigned)nx) return;
    const size_t nxy = (size_t)nx * ny;
    const size_t ro = (size_t)k * nxy + (size_t)j * nx;
    const TP* __restrict__ pr = a.p + ro;
    const TP* __restrict__ py = (j > 0) ? pr - nx : pr + (size_t)(ny - 1) * nx;   // j-1, wrapped
    const TP* __restrict__ pz = (k > 0) ? pr - nxy : pr;                           // unused at k = 0
    const unsigned im = (i > 0) ? i - 1 : (unsigned)nx - 1;
    const VP pc = *reinterpret_cast<const VP*>(pr + i);
    const TP pxm = pr[im];
    const VP pyv = *reinterpret_cast<const VP*>(py + i);
    const VP pzv = *reinterpret_cast<const VP*>(pz + i);
    TIO* __restrict__ u = a.u + ro;
    TIO* __restrict__ v = a.v + ro;
    TIO* __restrict__ w = a.w + ro;
    const V uo = *reinterpret_cast<const V*>(u + i);
    const V vo = *reinterpret_cast<const V*>(v + i);
    const V wo = *reinterpret_cast<const V*>(w + i);
    const TIO bk = a.bk[k], gk = a.gk[k];
    V un, vn, wn;
    un.x = (a.bcx == FSEI_BC_WALL && i == 0) ? (TIO)0 : uo.x + a.cx * ((TIO)pc.x - (TIO)pxm);
    un.y = uo.y + a.cx * ((TIO)pc.y - (TIO)pc.x);
    const bool v0 = a.bcy == FSEI_BC_WALL && j == 0;
    vn.x = v0 ? (TIO)0 : vo.x + a.cy * ((TIO)pc.x - (TIO)pyv.x);
    vn.y = v0 ? (TIO)0 : vo.y + a.cy * ((TIO)pc.y - (TIO)pyv.y);
    wn.x = (k == 0) ? (TIO)0 : wo.x + a.sw * (bk * (TIO)pc.x - gk * (TIO)pzv.x);
    wn.y = (k == 0) ? (TIO)0 : wo.y + a.sw * (bk * (TIO)pc.y - gk * (TIO)pzv.y);
    *reinterpret_cast<V*>(u + i) = un;
    *reinterpret_cast<V*>(v + i) = vn;
    *reinterpret_cast<V*>(w + i) = wn;
}

// ---------------------------------------------------------------------------
// FP64 residual norm of the refinement, r = (f - mean) - L p: per-block
// (sum r^2, sum r, sum dz_k p) partials.  The third sum is the volume
// integral of the iterate (over dx dy): the residual is blind to constants,
// so this is what lets a correction pin the V-mean of p in FP64.  Lanes own
// two adjacent x-cells (16-byte accesses), workgroups RJ rows of one
// z-plane, tiles plane-fastest (the k-1 rows of p were read by the previous
// workgroup on the same XCD); the j-1 / j+1 rows rotate through registers.
// ---------------------------------------------------------------------------
template <typename TPP>
struct ResArgs {
    int nx, ny, nz, bcx, bcy;
    const double* f;
    const TPP* p;         // pressure iterate (FP64, or the first FP32 solve)
    double idx2, idy2;
    const double* za;
    const double* zc;
    const double* scal;   // scal[0] = removed mean
    const double* dz;     // cell widths dz_k (third partial)
    double* partials;
};

// two adjacent values of T as a double2
template <typename T>
__device__ __forceinline__ double2 ld2d(const T* q) {
    const auto v = *reinterpret_cast<const typename Vec2T<T>::type*>(q);
    return make_double2((double)v.x, (double)v.y);
}

template <int NT, int RJ, typename TPP, int RB = 2>   // RB: rows per load batch
__global__ __launch_bounds__(NT) void k_resid_pairs(ResArgs<TPP> a) {
    static_assert(RJ % RB == 0, "whole batches");
    __shared__ double sred[3 * (NT / 64)];
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int b = (int)xcd_remap(blockIdx.x, gridDim.x);
    const int jt = b / nz;
    const int k = b - jt * nz;
    const int j0 = jt * RJ;
    const size_t nxy = (size_t)nx * ny;
    const TPP* __restrict__ pk = a.p + (size_t)k * nxy;
    const TPP* __restrict__ pkm = (k > 0) ? pk - nxy : pk;
    const TPP* __restrict__ pkp = (k + 1 < nz) ? pk + nxy : pk;
    const double* __restrict__ fk = a.f + (size_t)k * nxy;
    const double czm = (k > 0) ? a.za[k] : 0.0, czp = (k + 1 < nz) ? a.zc[k] : 0.0;
    const bool hzm = k > 0, hzp = k + 1 < nz;
    const bool pery = a.bcy == FSEI_BC_PERIODIC, perx = a.bcx == FSEI_BC_PERIODIC;
    const double mean = a.scal[0];
    double ss = 0.0, s1 = 0.0, sp = 0.0;
    for (int c = threadIdx.x; 2 * c < nx; c += NT) {
        const unsigned i = 2u * (unsigned)c;
        // x neighbours of the pair: i - 1 and i + 2 (wrapped)
        const unsigned im = (i > 0) ? i - 1 : (unsigned)nx - 1;
        const unsigned ip = (i + 2 < (unsigned)nx) ? i + 2 : 0u;
        const bool him = (i > 0) || perx, hip = (i + 2 < (unsigned)nx) || perx;
        const int jm0 = (j0 > 0) ? j0 - 1 : ny - 1;
        double2 pm = ld2d(pk + (size_t)jm0 * nx + i);
        double2 pc = ld2d(pk + (size_t)j0 * nx + i);
#pragma unroll
        for (int l0 = 0; l0 < RJ; l0 += RB) {
            double2 pn[RB], pzm[RB], pzp[RB], fc[RB];
            double pxm[RB], pxp[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int j = j0 + l0 + r;
                const size_t ro = (size_t)j * nx;
                const int jn = (j + 1 < ny) ? j + 1 : 0;
                pn[r] = ld2d(pk + (size_t)jn * nx + i);
                pxm[r] = (double)pk[ro + im];
                pxp[r] = (double)pk[ro + ip];
                pzm[r] = ld2d(pkm + ro + i);
                pzp[r] = ld2d(pkp + ro + i);
                fc[r] = *reinterpret_cast<const double2*>(fk + ro + i);
            }
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int j = j0 + l0 + r;
                const bool hym = (j > 0) || pery, hyp = (j + 1 < ny) || pery;
                // cell i: x neighbours i+1 (= pc.y) and i-1; cell i+1: i+2 and i
                const double lx0 = (pc.y - pc.x) + (him ? pxm[r] - pc.x : 0.0);
                const double lx1 = (hip ? pxp[r] - pc.y : 0.0) + (pc.x - pc.y);
                const double ly0 = (hyp ? pn[r].x - pc.x : 0.0) + (hym ? pm.x - pc.x : 0.0);
                const double ly1 = (hyp ? pn[r].y - pc.y : 0.0) + (hym ? pm.y - pc.y : 0.0);
                const double lz0 = (hzp ? czp * (pzp[r].x - pc.x) : 0.0) + (hzm ? czm * (pzm[r].x - pc.x) : 0.0);
                const double lz1 = (hzp ? czp * (pzp[r].y - pc.y) : 0.0) + (hzm ? czm * (pzm[r].y - pc.y) : 0.0);
                const double r0 = (fc[r].x - mean) - (lx0 * a.idx2 + ly0 * a.idy2 + lz0);
                const double r1 = (fc[r].y - mean) - (lx1 * a.idx2 + ly1 * a.idy2 + lz1);
                ss += r0 * r0 + r1 * r1;
                s1 += r0 + r1;
                sp += pc.x + pc.y;
                pm = pc;
                pc = pn[r];
            }
        }
    }
    double s2 = a.dz[k] * sp;   // every row of the block is in plane k
    block_sum3<NT>(ss, s1, s2, sred);
    if (threadIdx.x == 0) {
        a.partials[3 * blockIdx.x] = ss;
        a.partials[3 * blockIdx.x + 1] = s1;
        a.partials[3 * blockIdx.x + 2] = s2;
    }
}

// ---------------------------------------------------------------------------
// Gradient correction fused with the FP64 residual norm of the refinement's
// current pressure iterate: u += cx (g_i - g_{i-1}), v += cy (g_j - g_{j-1}),
// w += sw (bk_k g_k - gk_k g_{k-1}) with g = p (or, DELTA, with g = the last
// correction c, applied on top of an earlier update), and the partials
// (sum r^2, sum r, 0) of r = (f - mean) - L p.  Pair tiling as
// k_resid_pairs.  The convergence check of the last correction then costs no
// pass of its own.
// ---------------------------------------------------------------------------
struct GradResArgs {
    int nx, ny, nz, bcx, bcy;
    double* u;
    double* v;
    double* w;
    const double* p;      // current iterate (residual; gradient unless DELTA)
    const float* c;       // DELTA: the correction whose gradient is applied
    double cx, cy, sw;
    const double* bk;
    const double* gk;
    const double* f;
    double idx2, idy2;
    const double* za;
    const double* zc;
    const double* scal;   // scal[0] = removed mean
    double* partials;
};

template <int NT, int RJ, bool DELTA>
__global__ __launch_bounds__(NT) void k_grad_resid(GradResArgs a) {
    constexpr int RB = 2;   // rows per load batch (20 doubles per row in flight)
    static_assert(RJ % RB == 0, "whole batches");
    __shared__ double sred[3 * (NT / 64)];
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int b = (int)xcd_remap(blockIdx.x, gridDim.x);
    const int jt = b / nz;
    const int k = b - jt * nz;
    const int j0 = jt * RJ;
    const size_t nxy = (size_t)nx * ny;
    const size_t pl = (size_t)k * nxy;
    const double* __restrict__ pk = a.p + pl;
    const double* __restrict__ pkm = (k > 0) ? pk - nxy : pk;
    const double* __restrict__ pkp = (k + 1 < nz) ? pk + nxy : pk;
    const float* __restrict__ ck = DELTA ? a.c + pl : nullptr;
    const float* __restrict__ ckm = (DELTA && k > 0) ? ck - nxy : ck;
    const double* __restrict__ fk = a.f + pl;
    double* __restrict__ uk = a.u + pl;
    double* __restrict__ vk = a.v + pl;
    double* __restrict__ wk = a.w + pl;
    const double czm = (k > 0) ? a.za[k] : 0.0, czp = (k + 1 < nz) ? a.zc[k] : 0.0;
    const bool hzm = k > 0, hzp = k + 1 < nz;
    const bool pery = a.bcy == FSEI_BC_PERIODIC, perx = a.bcx == FSEI_BC_PERIODIC;
    const bool wallx = !perx, wally = !pery;
    const double mean = a.scal[0];
    const double bkk = a.bk[k], gkk = a.gk[k];
    double ss = 0.0, s1 = 0.0;
    for (int c = threadIdx.x; 2 * c < nx; c += NT) {
        const unsigned i = 2u * (unsigned)c;
        const unsigned im = (i > 0) ? i - 1 : (unsigned)nx - 1;
        const unsigned ip = (i + 2 < (unsigned)nx) ? i + 2 : 0u;
        const bool him = (i > 0) || perx, hip = (i + 2 < (unsigned)nx) || perx;
        const int jm0 = (j0 > 0) ? j0 - 1 : ny - 1;
        double2 pm = ld2d(pk + (size_t)jm0 * nx + i);
        double2 pc = ld2d(pk + (size_t)j0 * nx + i);
        double2 cm = make_double2(0.0, 0.0);
        if constexpr (DELTA) cm = ld2d(ck + (size_t)jm0 * nx + i);
#pragma unroll
        for (int l0 = 0; l0 < RJ; l0 += RB) {
            double2 pn[RB], pzm[RB], pzp[RB], fc[RB], uo[RB], vo[RB], wo[RB], cc[RB], czk[RB];
            double pxm[RB], pxp[RB], cxm[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int j = j0 + l0 + r;
                const size_t ro = (size_t)j * nx;
                const int jn = (j + 1 < ny) ? j + 1 : 0;
                pn[r] = ld2d(pk + (size_t)jn * nx + i);
                pxm[r] = pk[ro + im];
                pxp[r] = pk[ro + ip];
                pzm[r] = ld2d(pkm + ro + i);
                pzp[r] = ld2d(pkp + ro + i);
                fc[r] = ld2d(fk + ro + i);
                uo[r] = ld2d(uk + ro + i);
                vo[r] = ld2d(vk + ro + i);
                wo[r] = ld2d(wk + ro + i);
                if constexpr (DELTA) {
                    cc[r] = ld2d(ck + ro + i);
                    cxm[r] = (double)ck[ro + im];
                    czk[r] = ld2d(ckm + ro + i);
                }
            }
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int j = j0 + l0 + r;
                const size_t ro = (size_t)j * nx;
                const bool hym = (j > 0) || pery, hyp = (j + 1 < ny) || pery;
                // residual of the current iterate (as k_resid_pairs)
                const double lx0 = (pc.y - pc.x) + (him ? pxm[r] - pc.x : 0.0);
                const double lx1 = (hip ? pxp[r] - pc.y : 0.0) + (pc.x - pc.y);
                const double ly0 = (hyp ? pn[r].x - pc.x : 0.0) + (hym ? pm.x - pc.x : 0.0);
                const double ly1 = (hyp ? pn[r].y - pc.y : 0.0) + (hym ? pm.y - pc.y : 0.0);
                const double lz0 = (hzp ? czp * (pzp[r].x - pc.x) : 0.0) + (hzm ? czm * (pzm[r].x - pc.x) : 0.0);
                const double lz1 = (hzp ? czp * (pzp[r].y - pc.y) : 0.0) + (hzm ? czm * (pzm[r].y - pc.y) : 0.0);
                const double r0 = (fc[r].x - mean) - (lx0 * a.idx2 + ly0 * a.idy2 + lz0);
                const double r1 = (fc[r].y - mean) - (lx1 * a.idx2 + ly1 * a.idy2 + lz1);
                ss += r0 * r0 + r1 * r1;
                s1 += r0 + r1;
                // gradient of g = p, or of the correction c
                const double2 gc = DELTA ? cc[r] : pc;
                const double2 gm = DELTA ? cm : pm;
                const double gxm = DELTA ? cxm[r] : pxm[r];
                const double2 gz = DELTA ? czk[r] : pzm[r];
                double2 un, vn, wn;
                un.x = (wallx && i == 0) ? 0.0 : uo[r].x + a.cx * (gc.x - gxm);
                un.y = uo[r].y + a.cx * (gc.y - gc.x);
                const bool v0 = wally && j == 0;
                vn.x = v0 ? 0.0 : vo[r].x + a.cy * (gc.x - gm.x);
                vn.y = v0 ? 0.0 : vo[r].y + a.cy * (gc.y - gm.y);
                wn.x = (k == 0) ? 0.0 : wo[r].x + a.sw * (bkk * gc.x - gkk * gz.x);
                wn.y = (k == 0) ? 0.0 : wo[r].y + a.sw * (bkk * gc.y - gkk * gz.y);
                *reinterpret_cast<double2*>(uk + ro + i) = un;
                *reinterpret_cast<double2*>(vk + ro + i) = vn;
                *reinterpret_cast<double2*>(wk + ro + i) = wn;
                pm = pc;
                pc = pn[r];
                if constexpr (DELTA) cm = cc[r];
            }
            // keep the next batch's loads after this batch's stores (bounds
            // the registers to one batch)
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    double s2 = 0.0;
    block_sum3<NT>(ss, s1, s2, sred);
    if (threadIdx.x == 0) {
        a.partials[3 * blockIdx.x] = ss;
        a.partials[3 * blockIdx.x + 1] = s1;
        a.partials[3 * blockIdx.x + 2] = 0.0;
    }
}

// out = (double) in, n values (grid-stride)
__global__ __launch_bounds__(256) void k_widen(const float* __restrict__ in, double* __restrict__ out, size_t n) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        out[i] = (double)in[i];
}

// deterministic sum of the per-block partial triples: one workgroup of NT
// threads, 8 triples in flight per thread, fixed summation order; optionally
// also mean_out = (third sum) * mean_scale
template <int NT>
__global__ __launch_bounds__(NT) void k_sum_partials(const double* part, int nblk, double* out, double* mean_out,
                                                    double mean_scale) {
    __shared__ double sh[3 * (NT / 64)];
    double a = 0.0, b = 0.0, c = 0.0;
    for (int t0 = threadIdx.x; t0 < nblk; t0 += 8 * NT) {
        double v[8][3];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int t = t0 + r * NT;
#pragma unroll
            for (int q = 0; q < 3; ++q) v[r][q] = (t < nblk) ? part[3 * t + q] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            a += v[r][0];
            b += v[r][1];
            c += v[r][2];
        }
    }
    block_sum3<NT>(a, b, c, sh);
    if (threadIdx.x == 0) {
        out[0] = a;
        out[1] = b;
        out[2] = c;
        if (mean_out) *mean_out = c * mean_scale;
    }
}

// first stage of the two-stage sum: workgroup g sums the triples
// [g * chunk, min(nblk, (g + 1) * chunk)) in a fixed order into grp[3 g ..]
__global__ __launch_bounds__(256) void k_sum_partials_grp(const double* part, int nblk, int chunk, double* grp) {
    __shared__ double sh[3 * 4];
    const int lo = blockIdx.x * chunk;
    const int hi = (lo + chunk < nblk) ? lo + chunk : nblk;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int t0 = lo + (int)threadIdx.x; t0 < hi; t0 += 4 * 256) {
        double v[4][3];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int t = t0 + r * 256;
#pragma unroll
            for (int q = 0; q < 3; ++q) v[r][q] = (t < hi) ? part[3 * t + q] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            a += v[r][0];
            b += v[r][1];
            c += v[r][2];
        }
    }
    block_sum3<256>(a, b, c, sh);
    if (threadIdx.x == 0) {
        grp[3 * blockIdx.x] = a;
        grp[3 * blockIdx.x + 1] = b;
        grp[3 * blockIdx.x + 2] = c;
    }
}

}  // namespace dev
}  // namespace fsei
