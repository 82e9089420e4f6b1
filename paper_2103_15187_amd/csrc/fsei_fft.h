// Batched mixed-radix (8/4/3/2) Stockham FFT in LDS for gfx950.
//
// A workgroup transforms `nseq` complex sequences of length N that sit in LDS
// as split real/imaginary arrays (sequence s, element n at logical index
// s*N + n).  Each radix-R stage reads R inputs at stride N/R, applies the
// twiddles exp(SIGN 2 pi i t / N), does a length-R DFT in registers and writes
// the outputs to their self-sorting positions, so the result is in natural
// order without a bit-reversal pass.  A stage is done in place: every thread
// first gathers all of its butterflies into registers, then the workgroup
// synchronises, then every thread scatters.
#pragma once

#include <hip/hip_runtime.h>

#include "fsei_plan.h"

namespace fsei {
namespace dev {

// LDS index with one pad slot every 16 elements (breaks the power-of-two
// strides of the scatter into distinct banks).
__device__ __forceinline__ int lp(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int lds_elems(int e) { return e + (e >> 4) + 1; }

template <typename T>
__device__ __forceinline__ void cmul(T& ar, T& ai, T br, T bi) {
    const T t = ar * br - ai * bi;
    ai = ar * bi + ai * br;
    ar = t;
}

// ---- length-R DFTs in registers, y_q = sum_r x_r exp(SIGN 2 pi i r q / R)
template <typename T, int SIGN>
__device__ __forceinline__ void dft2(T* xr, T* xi) {
    const T ar = xr[0] + xr[1], ai = xi[0] + xi[1];
    xr[1] = xr[0] - xr[1];
    xi[1] = xi[0] - xi[1];
    xr[0] = ar;
    xi[0] = ai;
}

template <typename T, int SIGN>
__device__ __forceinline__ void dft4v(T x0r, T x0i, T x1r, T x1i, T x2r, T x2i, T x3r, T x3i,
                                      T* yr, T* yi) {
    const T ar = x0r + x2r, ai = x0i + x2i;
    const T br = x0r - x2r, bi = x0i - x2i;
    const T cr = x1r + x3r, ci = x1i + x3i;
    const T dr = x1r - x3r, di = x1i - x3i;
    yr[0] = ar + cr;
    yi[0] = ai + ci;
    yr[2] = ar - cr;
    yi[2] = ai - ci;
    // y1 = b + SIGN i d, y3 = b - SIGN i d
    yr[1] = br - SIGN * di;
    yi[1] = bi + SIGN * dr;
    yr[3] = br + SIGN * di;
    yi[3] = bi - SIGN * dr;
}

template <typename T, int SIGN>
__device__ __forceinline__ void dft4(T* xr, T* xi) {
    T yr[4], yi[4];
    dft4v<T, SIGN>(xr[0], xi[0], xr[1], xi[1], xr[2], xi[2], xr[3], xi[3], yr, yi);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        xr[q] = yr[q];
        xi[q] = yi[q];
    }
}

template <typename T, int SIGN>
__device__ __forceinline__ void dft8(T* xr, T* xi) {
    T er[4], ei[4], orr[4], oi[4];
    dft4v<T, SIGN>(xr[0], xi[0], xr[2], xi[2], xr[4], xi[4], xr[6], xi[6], er, ei);
    dft4v<T, SIGN>(xr[1], xi[1], xr[3], xi[3], xr[5], xi[5], xr[7], xi[7], orr, oi);
    const T h = (T)0.70710678118654752440084436210484903928;
    // w^q O_q with w = exp(SIGN i pi / 4)
    T tr[4], ti[4];
    tr[0] = orr[0];
    ti[0] = oi[0];
    tr[1] = h * (orr[1] - SIGN * oi[1]);
    ti[1] = h * (oi[1] + SIGN * orr[1]);
    tr[2] = -SIGN * oi[2];
    ti[2] = SIGN * orr[2];
    tr[3] = h * (-orr[3] - SIGN * oi[3]);
    ti[3] = h * (-oi[3] + SIGN * orr[3]);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        xr[q] = er[q] + tr[q];
        xi[q] = ei[q] + ti[q];
        xr[q + 4] = er[q] - tr[q];
        xi[q + 4] = ei[q] - ti[q];
    }
}

template <typename T, int SIGN>
__device__ __forceinline__ void dft3(T* xr, T* xi) {
    const T s3 = (T)0.86602540378443864676372317075293618347;
    const T tr = xr[1] + xr[2], ti = xi[1] + xi[2];
    const T ur = xr[1] - xr[2], ui = xi[1] - xi[2];
    const T mr = xr[0] - (T)0.5 * tr, mi = xi[0] - (T)0.5 * ti;
    xr[0] = xr[0] + tr;
    xi[0] = xi[0] + ti;
    xr[1] = mr - SIGN * s3 * ui;
    xi[1] = mi + SIGN * s3 * ur;
    xr[2] = mr + SIGN * s3 * ui;
    xi[2] = mi - SIGN * s3 * ur;
}

template <typename T, int R, int SIGN>
__device__ __forceinline__ void dftR(T* xr, T* xi) {
    if constexpr (R == 2) dft2<T, SIGN>(xr, xi);
    else if constexpr (R == 3) dft3<T, SIGN>(xr, xi);
    else if constexpr (R == 4) dft4<T, SIGN>(xr, xi);
    else dft8<T, SIGN>(xr, xi);
}

// One Stockham stage of radix R over all nseq sequences.  MAXB bounds the
// butterflies per thread: nseq*N/R <= MAXB*blockDim.x.
template <typename T, int R, int MAXB, int SIGN>
__device__ __forceinline__ void fft_stage(T* __restrict__ re, T* __restrict__ im, int N, int nseq, int Ns,
                                          const T* __restrict__ twc, const T* __restrict__ tws) {
    const int NR = N / R;
    const int nb = nseq * NR;
    const int tstep = N / (Ns * R);
    T vr[MAXB][R], vi[MAXB][R];
    int dst[MAXB];
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        const int w = threadIdx.x + b * blockDim.x;
        dst[b] = -1;
        if (w < nb) {
            const int s = w / NR;
            const int j = w - s * NR;
            const int k = j % Ns;
            const int base = s * N;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                vr[b][r] = re[lp(base + j + r * NR)];
                vi[b][r] = im[lp(base + j + r * NR)];
            }
            if (Ns > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    const int t = k * r * tstep;
                    cmul(vr[b][r], vi[b][r], twc[t], (T)SIGN * tws[t]);
                }
            }
            dftR<T, R, SIGN>(vr[b], vi[b]);
            dst[b] = base + (j - k) * R + k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        if (dst[b] >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                re[lp(dst[b] + r * Ns)] = vr[b][r];
                im[lp(dst[b] + r * Ns)] = vi[b][r];
            }
        }
    }
    __syncthreads();
}

__host__ __device__ constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }

// Full transform of nseq sequences (nseq*N <= EMAX) with NTHR threads.
template <typename T, int EMAX, int NTHR, int SIGN>
__device__ void fft_lds(T* re, T* im, int N, int nseq, const FftPlan& pl, const T* __restrict__ twc,
                        const T* __restrict__ tws) {
    int Ns = 1;
    for (int st = 0; st < pl.nstages; ++st) {
        const int R = pl.radix[st];
        if (R == 8)
            fft_stage<T, 8, cdiv(EMAX, NTHR * 8), SIGN>(re, im, N, nseq, Ns, twc, tws);
        else if (R == 4)
            fft_stage<T, 4, cdiv(EMAX, NTHR * 4), SIGN>(re, im, N, nseq, Ns, twc, tws);
        else if (R == 2)
            fft_stage<T, 2, cdiv(EMAX, NTHR * 2), SIGN>(re, im, N, nseq, Ns, twc, tws);
        else
            fft_stage<T, 3, cdiv(EMAX, NTHR * 3), SIGN>(re, im, N, nseq, Ns, twc, tws);
        Ns *= R;
    }
}

}  // namespace dev
}  // namespace fsei
