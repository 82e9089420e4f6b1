// HIP kernels of the pressure projection for gfx950 (MI355X).
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
//
// Transforms (paper, Program summary: FFTW in the homogeneous directions):
// two real lines a, b travel as one complex sequence z = a + i b through a
// length-N FFT.  Walls use the DCT-II basis cos(pi q (i+1/2)/N), computed from
// the even/odd reordering v_n = x_{2n}, v_{N-1-n} = x_{2n+1} and a post-twiddle
// exp(-i pi q / 2N) (Makhoul's method); periodic directions use the real DFT
// in half-complex layout (real parts at rows 0..N/2, imaginary parts of mode
// m at row N-m).  Both inverses are unnormalised (they return N times the
// input); the z solve folds in the factor 1/(nx ny).
#pragma once

#include <hip/hip_runtime.h>

#include "fsei_fft.h"
#include "fsei_plan.h"

namespace fsei {
namespace dev {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
// position of element i in the even/odd reordered sequence (walls)
__device__ __forceinline__ int mk_pos(int i, int N) { return (i & 1) ? N - 1 - (i >> 1) : (i >> 1); }

// deterministic block sum of two values (result valid in thread 0)
template <int NTHR>
__device__ __forceinline__ void block_sum2(double& a, double& b, double* sh) {
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        sh[2 * wid] = a;
        sh[2 * wid + 1] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0.0, sb = 0.0;
        for (int w = 0; w < NTHR / 64; ++w) {
            sa += sh[2 * w];
            sb += sh[2 * w + 1];
        }
        a = sa;
        b = sb;
    }
    __syncthreads();
}

// forward post-processing of pair s: the two real outputs at row m
template <typename T>
__device__ __forceinline__ void post_fwd(const T* re, const T* im, int base, int N, int m, int bc,
                                         const T* __restrict__ dctc, const T* __restrict__ dcts, T& xa,
                                         T& xb) {
    const T half = (T)0.5;
    if (bc == FSEI_BC_WALL) {
        const int mm = (m == 0) ? 0 : N - m;
        const T zr = re[lp(base + m)], zi = im[lp(base + m)];
        const T cr = re[lp(base + mm)], ci = im[lp(base + mm)];
        const T ar = (zr + cr) * half, ai = (zi - ci) * half;
        const T br = (zi + ci) * half, bi = (cr - zr) * half;
        const T wr = dctc[m], wi = -dcts[m];
        xa = wr * ar - wi * ai;
        xb = wr * br - wi * bi;
    } else {
        if (2 * m <= N) {
            const int mm = (m == 0) ? 0 : N - m;
            xa = (re[lp(base + m)] + re[lp(base + mm)]) * half;
            xb = (im[lp(base + m)] + im[lp(base + mm)]) * half;
        } else {
            const int q = N - m;
            xa = (im[lp(base + q)] - im[lp(base + m)]) * half;
            xb = (re[lp(base + m)] - re[lp(base + q)]) * half;
        }
    }
}

// inverse pre-processing: complex input Z[m] of the pair from the rows m and
// N-m of the two transformed lines
template <typename T>
__device__ __forceinline__ void pre_inv(int N, int m, int bc, T xam, T xanm, T xbm, T xbnm,
                                        const T* __restrict__ dctc, const T* __restrict__ dcts, T& zr, T& zi) {
    if (bc == FSEI_BC_WALL) {
        if (m == 0) {
            xanm = (T)0;
            xbnm = (T)0;
        }
        const T c = dctc[m], s = dcts[m];
        const T var = c * xam + s * xanm, vai = s * xam - c * xanm;
        const T vbr = c * xbm + s * xbnm, vbi = s * xbm - c * xbnm;
        zr = var - vbi;
        zi = vai + vbr;
    } else {
        T ra, ia, rb, ib;
        if (2 * m <= N) {
            ra = xam;
            rb = xbm;
            const bool hasim = (m != 0) && (2 * m != N);
            ia = hasim ? xanm : (T)0;
            ib = hasim ? xbnm : (T)0;
        } else {
            ra = xanm;
            rb = xbnm;
            ia = -xam;
            ib = -xbm;
        }
        zr = ra - ib;
        zi = ia + rb;
    }
}

// ---------------------------------------------------------------------------
// x forward: prologue (divergence / transposed gradient / residual / copy)
// fused with the forward x transform
// ---------------------------------------------------------------------------
enum { PRO_COPY = 0, PRO_DIV = 1, PRO_DIV_ADJ = 2, PRO_RESID = 3 };

template <typename TI, typename TO>
struct XFwdArgs {
    int nx, ny, nz, bcx, bcy, nseq;
    FftPlan fp;
    // prologue inputs
    const TI* u;
    const TI* v;
    const TI* w;
    const TI* gp;       // adjoint: dLoss/dp or null
    const double* f;    // COPY (double input) and RESID
    const double* p;    // RESID
    TI alpha, beta, idx, idy;
    const TI* zeta;     // coefficient of w_{k+1}
    const TI* eta;      // coefficient of w_k
    double idx2, idy2;  // RESID
    const double* za;   // RESID
    const double* zc;   // RESID
    const double* scal; // RESID: scal[0] = removed mean
    // outputs
    TO* out;
    double* out_f;      // optional FP64 copy of the prologue value
    double* partials;   // optional per-block (sum v^2, sum v)
    const TO* twc;
    const TO* tws;
    const TO* dctc;
    const TO* dcts;
};

template <typename TI, typename TO, int PRO>
__device__ __forceinline__ TI x_prologue(const XFwdArgs<TI, TO>& a, int k, int j, int i, size_t idx) {
    if constexpr (PRO == PRO_COPY) {
        return (TI)a.f[idx];
    } else if constexpr (PRO == PRO_RESID) {
        const int nx = a.nx, ny = a.ny, nz = a.nz;
        const size_t nxy = (size_t)nx * ny;
        const double* p = a.p;
        const double pc = p[idx];
        double lx = 0.0, ly = 0.0, lz = 0.0;
        if (i + 1 < nx) lx += p[idx + 1] - pc;
        else if (a.bcx == FSEI_BC_PERIODIC) lx += p[idx + 1 - nx] - pc;
        if (i >= 1) lx += p[idx - 1] - pc;
        else if (a.bcx == FSEI_BC_PERIODIC) lx += p[idx + nx - 1] - pc;
        if (j + 1 < ny) ly += p[idx + nx] - pc;
        else if (a.bcy == FSEI_BC_PERIODIC) ly += p[idx - (size_t)(ny - 1) * nx] - pc;
        if (j >= 1) ly += p[idx - nx] - pc;
        else if (a.bcy == FSEI_BC_PERIODIC) ly += p[idx + (size_t)(ny - 1) * nx] - pc;
        if (k + 1 < nz) lz += a.zc[k] * (p[idx + nxy] - pc);
        if (k >= 1) lz += a.za[k] * (p[idx - nxy] - pc);
        const double lap = lx * a.idx2 + ly * a.idy2 + lz;
        return (TI)((a.f[idx] - a.scal[0]) - lap);
    } else {
        const int nx = a.nx, ny = a.ny, nz = a.nz;
        const TI zero = (TI)0;
        const TI uc = (a.bcx == FSEI_BC_WALL && i == 0) ? zero : a.u[idx];
        const TI uh = (i + 1 < nx) ? a.u[idx + 1] : ((a.bcx == FSEI_BC_PERIODIC) ? a.u[idx + 1 - nx] : zero);
        const TI vc = (a.bcy == FSEI_BC_WALL && j == 0) ? zero : a.v[idx];
        const TI vh = (j + 1 < ny) ? a.v[idx + nx]
                                   : ((a.bcy == FSEI_BC_PERIODIC) ? a.v[idx - (size_t)(ny - 1) * nx] : zero);
        const TI wc = (k == 0) ? zero : a.w[idx];
        const TI wh = (k + 1 < nz) ? a.w[idx + (size_t)nx * ny] : zero;
        TI val = (uh - uc) * a.idx + (vh - vc) * a.idy + (a.zeta[k] * wh - a.eta[k] * wc);
        val *= a.alpha;
        if constexpr (PRO == PRO_DIV_ADJ) {
            if (a.gp) val += a.beta * a.gp[idx];
        }
        return val;
    }
}

template <typename TI, typename TO, int PRO, int EMAX, int NTHR>
__global__ __launch_bounds__(NTHR) void k_xfwd(XFwdArgs<TI, TO> a) {
    __shared__ TO sre[lds_elems(EMAX)];
    __shared__ TO sim[lds_elems(EMAX)];
    __shared__ double sred[2 * (NTHR / 64)];
    const int N = a.nx;
    const int nl = 2 * a.nseq;
    const long row0 = (long)blockIdx.x * nl;
    const long nrows = (long)a.ny * a.nz;
    double ss = 0.0, s1 = 0.0;
    for (int e = threadIdx.x; e < nl * N; e += NTHR) {
        const int l = e / N;
        const int i = e - l * N;
        const long row = row0 + l;
        TI val = (TI)0;
        if (row < nrows) {
            const int k = (int)(row / a.ny);
            const int j = (int)(row - (long)k * a.ny);
            const size_t idx = (size_t)row * N + i;
            val = x_prologue<TI, TO, PRO>(a, k, j, i, idx);
            if (a.out_f) a.out_f[idx] = (double)val;
            ss += (double)val * (double)val;
            s1 += (double)val;
        }
        const int s = l >> 1;
        const int n = (a.bcx == FSEI_BC_WALL) ? mk_pos(i, N) : i;
        if (l & 1) sim[lp(s * N + n)] = (TO)val;
        else sre[lp(s * N + n)] = (TO)val;
    }
    if (a.partials) {
        block_sum2<NTHR>(ss, s1, sred);
        if (threadIdx.x == 0) {
            a.partials[2 * blockIdx.x] = ss;
            a.partials[2 * blockIdx.x + 1] = s1;
        }
    } else {
        __syncthreads();
    }
    if (a.out == nullptr) return;   // norm-only pass (uniform over the block)
    fft_lds<TO, EMAX, NTHR, -1>(sre, sim, N, a.nseq, a.fp, a.twc, a.tws);
    for (int e = threadIdx.x; e < a.nseq * N; e += NTHR) {
        const int s = e / N;
        const int m = e - s * N;
        const long rowa = row0 + 2 * s;
        TO xa, xb;
        post_fwd<TO>(sre, sim, s * N, N, m, a.bcx, a.dctc, a.dcts, xa, xb);
        if (rowa < nrows) a.out[(size_t)rowa * N + m] = xa;
        if (rowa + 1 < nrows) a.out[(size_t)(rowa + 1) * N + m] = xb;
    }
}

// ---------------------------------------------------------------------------
// x inverse: unnormalised inverse x transform of row pairs; writes (STORE)
// or adds (ACC) the result into the output field
// ---------------------------------------------------------------------------
enum { EPI_STORE = 0, EPI_ACC = 1 };

template <typename T, typename TP>
struct XInvArgs {
    int nx, ny, nz, bcx, nseq;
    FftPlan fp;
    const T* in;
    TP* out;
    const T* twc;
    const T* tws;
    const T* dctc;
    const T* dcts;
};

template <typename T, typename TP, int EPI, int EMAX, int NTHR>
__global__ __launch_bounds__(NTHR) void k_xinv(XInvArgs<T, TP> a) {
    __shared__ T sre[lds_elems(EMAX)];
    __shared__ T sim[lds_elems(EMAX)];
    const int N = a.nx;
    const int nl = 2 * a.nseq;
    const long row0 = (long)blockIdx.x * nl;
    const long nrows = (long)a.ny * a.nz;
    for (int e = threadIdx.x; e < a.nseq * N; e += NTHR) {
        const int s = e / N;
        const int m = e - s * N;
        const int nm = (m == 0) ? 0 : N - m;
        const long rowa = row0 + 2 * s;
        T xam = 0, xanm = 0, xbm = 0, xbnm = 0;
        if (rowa < nrows) {
            xam = a.in[(size_t)rowa * N + m];
            xanm = a.in[(size_t)rowa * N + nm];
        }
        if (rowa + 1 < nrows) {
            xbm = a.in[(size_t)(rowa + 1) * N + m];
            xbnm = a.in[(size_t)(rowa + 1) * N + nm];
        }
        T zr, zi;
        pre_inv<T>(N, m, a.bcx, xam, xanm, xbm, xbnm, a.dctc, a.dcts, zr, zi);
        sre[lp(s * N + m)] = zr;
        sim[lp(s * N + m)] = zi;
    }
    __syncthreads();
    fft_lds<T, EMAX, NTHR, 1>(sre, sim, N, a.nseq, a.fp, a.twc, a.tws);
    for (int e = threadIdx.x; e < nl * N; e += NTHR) {
        const int l = e / N;
        const int i = e - l * N;
        const long row = row0 + l;
        if (row >= nrows) continue;
        const int s = l >> 1;
        const int n = (a.bcx == FSEI_BC_WALL) ? mk_pos(i, N) : i;
        const T val = (l & 1) ? sim[lp(s * N + n)] : sre[lp(s * N + n)];
        const size_t idx = (size_t)row * N + i;
        if constexpr (EPI == EPI_ACC) a.out[idx] += (TP)val;
        else a.out[idx] = (TP)val;
    }
}

// ---------------------------------------------------------------------------
// y transforms, in place, on tiles of TX = 2*nseq adjacent x-columns of one
// z-plane (each column pair is one complex sequence)
// ---------------------------------------------------------------------------
template <typename T>
struct YArgs {
    int nx, ny, nz, bcy, nseq, ntile;
    FftPlan fp;
    T* data;
    const T* twc;
    const T* tws;
    const T* dctc;
    const T* dcts;
};

template <typename T, int EMAX, int NTHR>
__global__ __launch_bounds__(NTHR) void k_yfwd(YArgs<T> a) {
    __shared__ T sre[lds_elems(EMAX)];
    __shared__ T sim[lds_elems(EMAX)];
    const int N = a.ny, nx = a.nx;
    const int TX = 2 * a.nseq;
    const int k = blockIdx.x / a.ntile;
    const int tile = blockIdx.x - k * a.ntile;
    const int i0 = tile * TX;
    T* __restrict__ d = a.data + (size_t)k * nx * N;
    for (int e = threadIdx.x; e < TX * N; e += NTHR) {
        const int j = e / TX;
        const int c = e - j * TX;
        const int i = i0 + c;
        const T val = (i < nx) ? d[(size_t)j * nx + i] : (T)0;
        const int n = (a.bcy == FSEI_BC_WALL) ? mk_pos(j, N) : j;
        const int s = c >> 1;
        if (c & 1) sim[lp(s * N + n)] = val;
        else sre[lp(s * N + n)] = val;
    }
    __syncthreads();
    fft_lds<T, EMAX, NTHR, -1>(sre, sim, N, a.nseq, a.fp, a.twc, a.tws);
    for (int e = threadIdx.x; e < a.nseq * N; e += NTHR) {
        const int m = e / a.nseq;
        const int s = e - m * a.nseq;
        T xa, xb;
        post_fwd<T>(sre, sim, s * N, N, m, a.bcy, a.dctc, a.dcts, xa, xb);
        const int i = i0 + 2 * s;
        if (i < nx) d[(size_t)m * nx + i] = xa;
        if (i + 1 < nx) d[(size_t)m * nx + i + 1] = xb;
    }
}

template <typename T, int EMAX, int NTHR>
__global__ __launch_bounds__(NTHR) void k_yinv(YArgs<T> a) {
    __shared__ T sre[lds_elems(EMAX)];
    __shared__ T sim[lds_elems(EMAX)];
    const int N = a.ny, nx = a.nx;
    const int TX = 2 * a.nseq;
    const int k = blockIdx.x / a.ntile;
    const int tile = blockIdx.x - k * a.ntile;
    const int i0 = tile * TX;
    T* __restrict__ d = a.data + (size_t)k * nx * N;
    for (int e = threadIdx.x; e < a.nseq * N; e += NTHR) {
        const int m = e / a.nseq;
        const int s = e - m * a.nseq;
        const int nm = (m == 0) ? 0 : N - m;
        const int i = i0 + 2 * s;
        T xam = 0, xanm = 0, xbm = 0, xbnm = 0;
        if (i < nx) {
            xam = d[(size_t)m * nx + i];
            xanm = d[(size_t)nm * nx + i];
        }
        if (i + 1 < nx) {
            xbm = d[(size_t)m * nx + i + 1];
            xbnm = d[(size_t)nm * nx + i + 1];
        }
        T zr, zi;
        pre_inv<T>(N, m, a.bcy, xam, xanm, xbm, xbnm, a.dctc, a.dcts, zr, zi);
        sre[lp(s * N + m)] = zr;
        sim[lp(s * N + m)] = zi;
    }
    __syncthreads();
    fft_lds<T, EMAX, NTHR, 1>(sre, sim, N, a.nseq, a.fp, a.twc, a.tws);
    for (int e = threadIdx.x; e < TX * N; e += NTHR) {
        const int j = e / TX;
        const int c = e - j * TX;
        const int i = i0 + c;
        if (i >= nx) continue;
        const int n = (a.bcy == FSEI_BC_WALL) ? mk_pos(j, N) : j;
        const int s = c >> 1;
        d[(size_t)j * nx + i] = (c & 1) ? sim[lp(s * N + n)] : sre[lp(s * N + n)];
    }
}

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
    __shared__ TC sh[7][NT];
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
    __syncthreads();
    sh[3][me] = al;
    sh[4][me] = be;
    sh[5][me] = ga;
    sh[6][me] = ph;
    __syncthreads();
    if (p == 0) {
        // Thomas on the P x P reduced system of line ln (c' into sh[5], d' into sh[6])
        TC cpr = 0, dpr = 0;
        for (int q = 0; q < P; ++q) {
            const int id = ln + q * TXL;
            const TC r = (TC)1 / (sh[4][id] - sh[3][id] * cpr);
            cpr = sh[5][id] * r;
            dpr = (sh[6][id] - sh[3][id] * dpr) * r;
            sh[5][id] = cpr;
            sh[6][id] = dpr;
        }
        TC x = 0;
        for (int q = P - 1; q >= 0; --q) {
            const int id = ln + q * TXL;
            x = sh[6][id] - sh[5][id] * x;
            sh[6][id] = x;
        }
    }
    __syncthreads();
    const TC XR = sh[6][me];
    const TC XL = (p > 0) ? sh[6][me - TXL] : (TC)0;
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
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y;
    const int k = blockIdx.z;
    const int nx = a.nx, ny = a.ny;
    if (i >= nx) return;
    const size_t idx = ((size_t)k * ny + j) * nx + i;
    const TIO pc = (TIO)a.p[idx];
    if (a.bcx == FSEI_BC_WALL && i == 0) {
        a.u[idx] = (TIO)0;
    } else {
        const TIO pm = (TIO)a.p[(i > 0) ? idx - 1 : idx + nx - 1];
        a.u[idx] += a.cx * (pc - pm);
    }
    if (a.bcy == FSEI_BC_WALL && j == 0) {
        a.v[idx] = (TIO)0;
    } else {
        const TIO pm = (TIO)a.p[(j > 0) ? idx - nx : idx + (size_t)(ny - 1) * nx];
        a.v[idx] += a.cy * (pc - pm);
    }
    if (k == 0) {
        a.w[idx] = (TIO)0;
    } else {
        const TIO pm = (TIO)a.p[idx - (size_t)nx * ny];
        a.w[idx] += a.sw * (a.bk[k] * pc - a.gk[k] * pm);
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
