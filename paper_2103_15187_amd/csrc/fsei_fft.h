// Batched mixed-radix (8/4/3/2) Stockham FFT in LDS for gfx950.
//
// A workgroup transforms `nseq` complex sequences of length N held in LDS as
// split real/imaginary arrays.  Element n of sequence s sits at
//     s * SP + n + n / 16,      SP = N + N / 16 + 1,
// i.e. one pad slot every 16 elements (breaks the power-of-two strides of a
// stage's scatter) and an odd stride between sequences (threads that walk
// across sequences at a fixed n hit different banks).  Each radix-R stage
// reads R inputs at stride N/R, applies the twiddles exp(SIGN 2 pi i t / N),
// does a length-R DFT in registers and writes the outputs to their
// self-sorting positions, so the result is in natural order without a
// bit-reversal pass.  A stage is done in place: every thread gathers all of
// its butterflies into registers, the workgroup synchronises, then scatters.
//
// When the length is a compile-time constant (NF > 0) the stage loop is
// unrolled with constant radices and strides, so no integer division remains.
#pragma once

#include <hip/hip_runtime.h>

#include "fsei_plan.h"

namespace fsei {
namespace dev {

// seq_stride, lds_elems and tile_nseq (the tile geometry) live in fsei_plan.h
template <int PS = kPadShift>
__device__ __forceinline__ int li(int s, int n, int SP) { return s * SP + n + (n >> PS); }

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
// butterflies per thread: nseq*N/R <= MAXB*blockDim.x.  N and Ns are
// compile-time constants when the caller's are.
template <typename T, int R, int MAXB, int SIGN, int NTHR, int PS = kPadShift>
__device__ __forceinline__ void fft_stage(T* __restrict__ re, T* __restrict__ im, int N, int SP, int nseq, int Ns,
                                          const T* __restrict__ twc, const T* __restrict__ tws) {
    const int NR = N / R;
    const int nb = nseq * NR;
    const int tstep = N / (Ns * R);
    T vr[MAXB][R], vi[MAXB][R];
    int dst[MAXB];
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        const int w = threadIdx.x + b * NTHR;
        dst[b] = -1;
        if (w < nb) {
            const int s = w / NR;
            const int j = w - s * NR;
            const int k = j % Ns;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int o = li<PS>(s, j + r * NR, SP);
                vr[b][r] = re[o];
                vi[b][r] = im[o];
            }
            if (Ns > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    const int t = k * r * tstep;
                    cmul(vr[b][r], vi[b][r], twc[t], (T)SIGN * tws[t]);
                }
            }
            dftR<T, R, SIGN>(vr[b], vi[b]);
            dst[b] = s * (1 << 20) + (j - k) * R + k;   // (sequence, position) packed
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        if (dst[b] >= 0) {
            const int s = dst[b] >> 20;
            const int pos = dst[b] & ((1 << 20) - 1);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int o = li<PS>(s, pos + r * Ns, SP);
                re[o] = vr[b][r];
                im[o] = vi[b][r];
            }
        }
    }
    __syncthreads();
}

__host__ __device__ constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }

// radix schedule shared with the host plan: 8s, then a 4 or a 2, then 3s
__host__ __device__ constexpr int pow2_part(int n) { return (n % 3 == 0) ? pow2_part(n / 3) : n; }
__host__ __device__ constexpr int num_stages(int n) {
    int m = pow2_part(n), c = 0;
    int r3 = 0;
    for (int t = n; t % 3 == 0; t /= 3) ++r3;
    while (m >= 8 && m % 8 == 0) {
        m /= 8;
        ++c;
    }
    if (m == 4 || m == 2) ++c;
    return c + r3;
}
__host__ __device__ constexpr int stage_radix(int n, int st) {
    int m = pow2_part(n), c = 0;
    while (m >= 8 && m % 8 == 0) {
        if (c == st) return 8;
        m /= 8;
        ++c;
    }
    if (m == 4 || m == 2) {
        if (c == st) return m;
        ++c;
    }
    return 3;
}

template <typename T, int EMAX, int NTHR, int SIGN, int NF, int ST, int NS, int PS = kPadShift>
__device__ __forceinline__ void fft_fixed(T* re, T* im, int nseq, const T* __restrict__ twc,
                                          const T* __restrict__ tws) {
    if constexpr (ST < num_stages(NF)) {
        constexpr int R = stage_radix(NF, ST);
        fft_stage<T, R, cdiv(EMAX, NTHR * R), SIGN, NTHR, PS>(re, im, NF, seq_stride(NF, PS), nseq, NS, twc, tws);
        fft_fixed<T, EMAX, NTHR, SIGN, NF, ST + 1, NS * R, PS>(re, im, nseq, twc, tws);
    }
}

// Full transform of nseq sequences (nseq*N <= EMAX) with NTHR threads.
template <typename T, int EMAX, int NTHR, int SIGN, int NF, int PS = kPadShift>
__device__ __forceinline__ void fft_lds(T* re, T* im, int N, int nseq, const FftPlan& pl,
                                        const T* __restrict__ twc, const T* __restrict__ tws) {
    if constexpr (NF > 0) {
        fft_fixed<T, EMAX, NTHR, SIGN, NF, 0, 1, PS>(re, im, nseq, twc, tws);
    } else {
        const int SP = seq_stride(N, PS);
        int Ns = 1;
        for (int st = 0; st < pl.nstages; ++st) {
            const int R = pl.radix[st];
            if (R == 8)
                fft_stage<T, 8, cdiv(EMAX, NTHR * 8), SIGN, NTHR, PS>(re, im, N, SP, nseq, Ns, twc, tws);
            else if (R == 4)
                fft_stage<T, 4, cdiv(EMAX, NTHR * 4), SIGN, NTHR, PS>(re, im, N, SP, nseq, Ns, twc, tws);
            else if (R == 2)
                fft_stage<T, 2, cdiv(EMAX, NTHR * 2), SIGN, NTHR, PS>(re, im, N, SP, nseq, Ns, twc, tws);
            else
                fft_stage<T, 3, cdiv(EMAX, NTHR * 3), SIGN, NTHR, PS>(re, im, N, SP, nseq, Ns, twc, tws);
            Ns *= R;
        }
    }
}

}  // namespace dev
}  // namespace fsei
