// Transform kernels of the pressure projection for gfx950 (MI355X): the x
// transforms (fused with the divergence / transposed-gradient / residual
// stencils on the way in and the pressure write or accumulation on the way
// out) and the y transforms.
//
// Transforms (paper, Program summary: FFTW in the homogeneous directions):
// two real lines a, b travel as one complex sequence z = a + i b through a
// length-N FFT.  Walls use the DCT-II basis cos(pi q (i+1/2)/N), computed from
// the even/odd reordering v_n = x_{2n}, v_{N-1-n} = x_{2n+1} and a post-twiddle
// exp(-i pi q / 2N) (Makhoul's method); periodic directions use the real DFT
// in half-complex layout (real parts at rows 0..N/2, imaginary parts of mode
// m at row N-m).  Both inverses are unnormalised (they return N times the
// input); the z solve folds in the factor 1/(nx ny).
//
// Every kernel has an optional compile-time length NF (0 = taken from the
// arguments): with NF fixed the FFT stages and all index arithmetic fold to
// constants.  Tile loops have compile-time trip counts and are unrolled, so
// a thread issues all loads of a batch before the first wait; addresses are
// 32-bit offsets from per-workgroup base pointers.
#pragma once

#include <hip/hip_runtime.h>

#include "fsei_fft.h"
#include "fsei_plan.h"

namespace fsei {
namespace dev {

// position of element i in the even/odd reordered sequence (walls)
__device__ __forceinline__ int mk_pos(int i, int N) { return (i & 1) ? N - 1 - (i >> 1) : (i >> 1); }

// Workgroups are handed to the 8 XCDs of the chip round-robin (workgroup i
// runs on XCD i % 8), and each XCD has its own L2.  This bijection of
// [0, n) gives XCD x a contiguous run of logical blocks, so blocks that
// touch neighbouring rows and planes (stencil halos) share an L2.
constexpr int kXcds = 8;
__device__ __forceinline__ long xcd_remap(long i, long n) {
    const long q = n / kXcds, r = n % kXcds;
    const long x = i % kXcds, t = i / kXcds;
    return x * q + (x < r ? x : r) + t;
}

// deterministic block sum of three values (result valid in thread 0)
template <int NTHR>
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c, double* sh) {
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
        c += __shfl_down(c, off, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        sh[3 * wid] = a;
        sh[3 * wid + 1] = b;
        sh[3 * wid + 2] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0.0, sb = 0.0, sc = 0.0;
        for (int w = 0; w < NTHR / 64; ++w) {
            sa += sh[3 * w];
            sb += sh[3 * w + 1];
            sc += sh[3 * w + 2];
        }
        a = sa;
        b = sb;
        c = sc;
    }
    __syncthreads();
}

// the length-N twiddle table exp(2 pi i t / N) in LDS (2 N values, in the
// kernel's dynamic LDS)
template <typename T>
__device__ __forceinline__ T* lds_twiddle_ptr() {
    extern __shared__ __align__(16) unsigned char dyn_lds[];
    return reinterpret_cast<T*>(dyn_lds);
}

// copies the twiddle table into LDS; visible after the next barrier.  The
// compile-time-length kernels call this after issuing their first field
// loads, so that the table's round trip overlaps theirs.
template <typename T, int NTHR>
__device__ __forceinline__ void stage_twiddles(T* twl, const T* __restrict__ twc, const T* __restrict__ tws, int N) {
    for (int t = threadIdx.x; t < N; t += NTHR) {
        twl[t] = twc[t];
        twl[N + t] = tws[t];
    }
}

// Compile-time length: the table is read into registers first (before the
// kernel's field loads are issued) and written to LDS after them, so its
// round trip overlaps theirs instead of preceding it.
template <typename T, int NTHR, int NF>
struct TwiddleRegs {
    static constexpr int IT = (NF + NTHR - 1) / NTHR;
    T c[IT], s[IT];
    __device__ __forceinline__ void load(const T* __restrict__ twc, const T* __restrict__ tws) {
#pragma unroll
        for (int r = 0; r < IT; ++r) {
            const int t = threadIdx.x + r * NTHR;
            c[r] = (t < NF) ? twc[t] : (T)0;
            s[r] = (t < NF) ? tws[t] : (T)0;
        }
    }
    __device__ __forceinline__ void store(T* twl) const {
#pragma unroll
        for (int r = 0; r < IT; ++r) {
            const int t = threadIdx.x + r * NTHR;
            if (t < NF) {
                twl[t] = c[r];
                twl[NF + t] = s[r];
            }
        }
    }
};

template <typename T, int NTHR>
__device__ __forceinline__ T* lds_twiddles(const T* __restrict__ twc, const T* __restrict__ tws, int N) {
    T* twl = lds_twiddle_ptr<T>();
    stage_twiddles<T, NTHR>(twl, twc, tws, N);
    return twl;
}

// forward post-processing of pair s: the two real outputs at row m
template <typename T, int PS = kPadShift>
__device__ __forceinline__ void post_fwd(const T* re, const T* im, int s, int SP, int N, int m, int bc,
                                         const T* __restrict__ dctc, const T* __restrict__ dcts, T& xa,
                                         T& xb) {
    const T half = (T)0.5;
    if (bc == FSEI_BC_WALL) {
        const int mm = (m == 0) ? 0 : N - m;
        const T zr = re[li<PS>(s, m, SP)], zi = im[li<PS>(s, m, SP)];
        const T cr = re[li<PS>(s, mm, SP)], ci = im[li<PS>(s, mm, SP)];
        const T ar = (zr + cr) * half, ai = (zi - ci) * half;
        const T br = (zi + ci) * half, bi = (cr - zr) * half;
        const T wr = dctc[m], wi = -dcts[m];
        xa = wr * ar - wi * ai;
        xb = wr * br - wi * bi;
    } else {
        if (2 * m <= N) {
            const int mm = (m == 0) ? 0 : N - m;
            xa = (re[li<PS>(s, m, SP)] + re[li<PS>(s, mm, SP)]) * half;
            xb = (im[li<PS>(s, m, SP)] + im[li<PS>(s, mm, SP)]) * half;
        } else {
            const int q = N - m;
            xa = (im[li<PS>(s, q, SP)] - im[li<PS>(s, m, SP)]) * half;
            xb = (re[li<PS>(s, m, SP)] - re[li<PS>(s, q, SP)]) * half;
        }
    }
}

// inverse pre-processing: complex input Z[m] of the pair from the rows m and
// N-m of the two transformed lines
template <typename T>
__device__ __forceinline__ void pre_inv_cs(int N, int m, int bc, T xam, T xanm, T xbm, T xbnm, T c, T s, T& zr,
                                           T& zi) {
    if (bc == FSEI_BC_WALL) {
        if (m == 0) {
            xanm = (T)0;
            xbnm = (T)0;
        }
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

// as pre_inv_cs with the twiddle pair read from the tables
template <typename T>
__device__ __forceinline__ void pre_inv(int N, int m, int bc, T xam, T xanm, T xbm, T xbnm,
                                        const T* __restrict__ dctc, const T* __restrict__ dcts, T& zr, T& zi) {
    T c = (T)1, s = (T)0;
    if (bc == FSEI_BC_WALL) {
        c = dctc[m];
        s = dcts[m];
    }
    pre_inv_cs<T>(N, m, bc, xam, xanm, xbm, xbnm, c, s, zr, zi);
}

// (k, j) of row j0 + l of plane k0 (rows wrap into the following planes)
__device__ __forceinline__ void row_kj(int k0, int j0, int l, int ny, int& k, int& j) {
    j = j0 + l;
    k = k0;
    if (j >= ny) {
        k += j / ny;
        j -= (j / ny) * ny;
    }
}

// ---------------------------------------------------------------------------
// Fixed-length full-tile paths.  The variants with NF > 0 are launched only
// when every tile is full (the host checks), so each thread's rows, columns
// and LDS slots are compile-time functions of its lane: loads and stores
// address a workgroup-uniform row pointer (scalar registers) plus the lane's
// 32-bit column, and every boundary test is either per row (uniform) or per
// lane and fixed for the whole launch.  No bounds test remains in the loops.
// ---------------------------------------------------------------------------

// neighbour rows of x-row (k, j): element offsets from the row and whether
// the neighbour takes part (a wall has no neighbour beyond it; an absent
// neighbour's offset is 0 so its load stays in bounds and is discarded)
struct RowNb {
    long yp, ym, zp, zm;
    bool hyp, hym, hzp, hzm;
};
__device__ __forceinline__ RowNb row_nb(int k, int j, int N, int ny, int nz, int bcy) {
    const bool per = bcy == FSEI_BC_PERIODIC;
    const long plane = (long)N * ny;
    RowNb r;
    r.hyp = (j + 1 < ny) || per;
    r.yp = (j + 1 < ny) ? (long)N : (per ? -(long)(ny - 1) * N : 0L);
    r.hym = (j >= 1) || per;
    r.ym = (j >= 1) ? -(long)N : (per ? (long)(ny - 1) * N : 0L);
    r.hzp = k + 1 < nz;
    r.zp = r.hzp ? plane : 0L;
    r.hzm = k >= 1;
    r.zm = r.hzm ? -plane : 0L;
    return r;
}

// x neighbours of column i: wrapped indices (always in [0, N)) and whether
// they take part
struct ColNb {
    unsigned i, ip, im;
    bool hip, him;
};
__device__ __forceinline__ ColNb col_nb(int i, int N, int bcx) {
    const bool per = bcx == FSEI_BC_PERIODIC;
    ColNb c;
    c.i = (unsigned)i;
    c.ip = (i + 1 < N) ? (unsigned)(i + 1) : 0u;
    c.im = (i >= 1) ? (unsigned)(i - 1) : (unsigned)(N - 1);
    c.hip = (i + 1 < N) || per;
    c.him = (i >= 1) || per;
    return c;
}

// forward post-processing from the four values at rows m and mm = (N - m) % N
// of one pair (selects instead of branches; same arithmetic as post_fwd)
template <typename T>
__device__ __forceinline__ void post_fwd_v(int bc, bool lo, T zr, T zi, T cr, T ci, T wr, T wi, T& xa, T& xb) {
    const T half = (T)0.5;
    if (bc == FSEI_BC_WALL) {
        const T ar = (zr + cr) * half, ai = (zi - ci) * half;
        const T br = (zi + ci) * half, bi = (cr - zr) * half;
        xa = wr * ar - wi * ai;
        xb = wr * br - wi * bi;
    } else {
        xa = lo ? (zr + cr) * half : (ci - zi) * half;
        xb = lo ? (zi + ci) * half : (zr - cr) * half;
    }
}

// whether the fixed y tile of EMAX elements and NTHR threads at length NF
// gives every thread whole column pairs on an even number of rows per pass
__host__ __device__ constexpr bool y_fixed_ok(int emax, int nthr, int nf, int ps = kPadShift) {
    return tile_nseq(emax, nf, ps) > 0 && nthr % tile_nseq(emax, nf, ps) == 0 &&
           nf % (nthr / tile_nseq(emax, nf, ps)) == 0 && (nthr / tile_nseq(emax, nf, ps)) % 2 == 0;
}

// LDS pad of the fixed-length y forward kernel: FP32 tiles run fastest with
// one pad slot per 64 elements, FP64 tiles with one per 16 (measured)
template <typename T>
constexpr int yfwd_pad() { return sizeof(T) == 4 ? 6 : kPadShift; }

// s_waitcnt immediates (vmcnt in bits 3:0 and 15:14, expcnt 6:4, lgkmcnt
// 11:8): wait until at most n vector-memory operations of this wave are
// outstanding; wait for this wave's LDS operations only
__device__ constexpr int imm_wait_vm(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }
__device__ constexpr int imm_wait_lgkm0() { return 15 | (3 << 14) | (7 << 4); }
// Workgroup barrier for LDS exchanges while direct global-to-LDS loads may
// still be in flight: this wave's LDS accesses complete, then the barrier,
// with no memory fence (a fence would wait for the direct loads too); the
// empty asm keeps the compiler from moving memory accesses across it.
__device__ __forceinline__ void sync_lds_nofence() {
    __builtin_amdgcn_s_waitcnt(imm_wait_lgkm0());
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// two adjacent values of a field as one vector access
template <typename T>
struct Vec2T;
template <>
struct Vec2T<double> {
    using type = double2;
};
template <>
struct Vec2T<float> {
    using type = float2;
};

// ---------------------------------------------------------------------------
// x forward: prologue (divergence / transposed gradient / residual / copy)
// fused with the forward x transform
// ---------------------------------------------------------------------------
// RESID: the FP64 residual (f - mean) - L p of an FP64 iterate p; RESID_F: of
// an FP32 iterate p32 (the first solve of the refinement), read as FP32 and
// evaluated in FP64
enum { PRO_COPY = 0, PRO_DIV = 1, PRO_DIV_ADJ = 2, PRO_RESID = 3, PRO_RESID_F = 5 };

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
    const float* p32;   // RESID_F
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
    double* partials;   // optional per-block (sum v^2, sum v, sum dzw_k v)
    const double* dzw;  // with partials: z weights of the third sum (dz_k), or null;
                        // RESID: the third sum is sum dzw_k p (the iterate, not r)
    const TO* twc;
    const TO* tws;
    const TO* dctc;
    const TO* dcts;
};

// the pressure iterate a residual prologue reads
template <int PRO, typename TI, typename TO>
__device__ __forceinline__ auto resid_iterate(const XFwdArgs<TI, TO>& a) {
    if constexpr (PRO == PRO_RESID_F) return a.p32;
    else return a.p;
}

// two adjacent values as a double2 (from double2 or float2)
__device__ __forceinline__ double2 pair_d(const double* q) { return *reinterpret_cast<const double2*>(q); }
__device__ __forceinline__ double2 pair_d(const float* q) {
    const float2 v = *reinterpret_cast<const float2*>(q);
    return make_double2((double)v.x, (double)v.y);
}

// The stencil value at cell (k, j, i); `o` is the cell's offset from the
// workgroup base `base` (first cell of its first row), so all accesses are
// 32-bit offsets from base pointers.
template <typename TI, typename TO, int PRO>
__device__ __forceinline__ TI x_prologue(const XFwdArgs<TI, TO>& a, size_t base, int k, int j, int i, int o,
                                         int N) {
    const int nx = N, ny = a.ny, nz = a.nz;
    const int nxy = nx * ny;
    if constexpr (PRO == PRO_COPY) {
        return (TI)a.f[base + o];
    } else if constexpr (PRO == PRO_RESID || PRO == PRO_RESID_F) {
        const auto* __restrict__ p = resid_iterate<PRO>(a) + base;
        const double pc = (double)p[o];
        double lx = 0.0, ly = 0.0, lz = 0.0;
        if (i + 1 < nx) lx += (double)p[o + 1] - pc;
        else if (a.bcx == FSEI_BC_PERIODIC) lx += (double)p[o + 1 - nx] - pc;
        if (i >= 1) lx += (double)p[o - 1] - pc;
        else if (a.bcx == FSEI_BC_PERIODIC) lx += (double)p[o + nx - 1] - pc;
        if (j + 1 < ny) ly += (double)p[o + nx] - pc;
        else if (a.bcy == FSEI_BC_PERIODIC) ly += (double)p[o - (ny - 1) * nx] - pc;
        if (j >= 1) ly += (double)p[o - nx] - pc;
        else if (a.bcy == FSEI_BC_PERIODIC) ly += (double)p[o + (ny - 1) * nx] - pc;
        if (k + 1 < nz) lz += a.zc[k] * ((double)p[o + nxy] - pc);
        if (k >= 1) lz += a.za[k] * ((double)p[o - nxy] - pc);
        const double lap = lx * a.idx2 + ly * a.idy2 + lz;
        return (TI)((a.f[base + o] - a.scal[0]) - lap);
    } else {
        const TI* __restrict__ u = a.u + base;
        const TI* __restrict__ v = a.v + base;
        const TI* __restrict__ w = a.w + base;
        const TI zero = (TI)0;
        const TI uc = (a.bcx == FSEI_BC_WALL && i == 0) ? zero : u[o];
        const TI uh = (i + 1 < nx) ? u[o + 1] : ((a.bcx == FSEI_BC_PERIODIC) ? u[o + 1 - nx] : zero);
        const TI vc = (a.bcy == FSEI_BC_WALL && j == 0) ? zero : v[o];
        const TI vh = (j + 1 < ny) ? v[o + nx] : ((a.bcy == FSEI_BC_PERIODIC) ? v[o - (ny - 1) * nx] : zero);
        const TI wc = (k == 0) ? zero : w[o];
        const TI wh = (k + 1 < nz) ? w[o + nxy] : zero;
        TI val = (uh - uc) * a.idx + (vh - vc) * a.idy + (a.zeta[k] * wh - a.eta[k] * wc);
        val *= a.alpha;
        if constexpr (PRO == PRO_DIV_ADJ) {
            if (a.gp) val += a.beta * a.gp[base + o];
        }
        return val;
    }
}

// x neighbours of the adjacent cells (i, i + 1), i even: i - 1 of the first
// and i + 2 of the second (wrapped; the flags say whether they take part)
struct PairNb {
    unsigned i, im, ip2;
    bool him, hip2;
};
__device__ __forceinline__ PairNb pair_nb(int i, int N, int bcx) {
    const bool per = bcx == FSEI_BC_PERIODIC;
    PairNb c;
    c.i = (unsigned)i;
    c.im = (i >= 1) ? (unsigned)(i - 1) : (unsigned)(N - 1);
    c.ip2 = (i + 2 < N) ? (unsigned)(i + 2) : 0u;
    c.him = (i >= 1) || per;
    c.hip2 = (i + 2 < N) || per;
    return c;
}

// The divergence / copy prologue for the two adjacent cells (i, i + 1) of a
// row, every field read as aligned pairs (the scalar x neighbour aside); the
// residual prologue of the compile-time-length path is written out in
// k_xfwd (it carries the iterate's rows down the tile)
template <typename TI, typename TO, int PRO>
__device__ __forceinline__ void x_prologue_pair(const XFwdArgs<TI, TO>& a, size_t ro, int k, const RowNb& rn,
                                                const PairNb& cn, TI& v0, TI& v1) {
    using V = typename Vec2T<TI>::type;
    if constexpr (PRO == PRO_COPY) {
        const double2 f = *reinterpret_cast<const double2*>(a.f + ro + cn.i);
        v0 = (TI)f.x;
        v1 = (TI)f.y;
    } else {
        const TI zero = (TI)0;
        const TI* __restrict__ u = a.u + ro;
        const TI* __restrict__ v = a.v + ro;
        const TI* __restrict__ w = a.w + ro;
        const V uc = *reinterpret_cast<const V*>(u + cn.i);
        const TI uh = u[cn.ip2];
        const V vc = *reinterpret_cast<const V*>(v + cn.i);
        const V vh = *reinterpret_cast<const V*>(v + rn.yp + cn.i);
        const V wc = *reinterpret_cast<const V*>(w + cn.i);
        const V wh = *reinterpret_cast<const V*>(w + rn.zp + cn.i);
        const TI zk = a.zeta[k], ek = a.eta[k];
        TI r0 = (uc.y - (cn.him ? uc.x : zero)) * a.idx + ((rn.hyp ? vh.x : zero) - (rn.hym ? vc.x : zero)) * a.idy +
                (zk * (rn.hzp ? wh.x : zero) - ek * (rn.hzm ? wc.x : zero));
        TI r1 = ((cn.hip2 ? uh : zero) - uc.y) * a.idx + ((rn.hyp ? vh.y : zero) - (rn.hym ? vc.y : zero)) * a.idy +
                (zk * (rn.hzp ? wh.y : zero) - ek * (rn.hzm ? wc.y : zero));
        r0 *= a.alpha;
        r1 *= a.alpha;
        if constexpr (PRO == PRO_DIV_ADJ) {
            if (a.gp) {
                const V g = *reinterpret_cast<const V*>(a.gp + ro + cn.i);
                r0 += a.beta * g.x;
                r1 += a.beta * g.y;
            }
        }
        v0 = r0;
        v1 = r1;
    }
}

template <typename TI, typename TO, int PRO, int EMAX, int NTHR, int NF>
__global__ __launch_bounds__(NTHR) void k_xfwd(XFwdArgs<TI, TO> a) {
    __shared__ TO sre[lds_elems(EMAX)];
    __shared__ TO sim[lds_elems(EMAX)];
    __shared__ double sred[3 * (NTHR / 64)];
    constexpr int NSF = NF > 0 ? tile_nseq(EMAX, NF) : 0;   // pairs per tile, fixed path
    const int N = NF > 0 ? NF : a.nx;
    const int SP = seq_stride(N);
    const int nseq = NF > 0 ? NSF : a.nseq;
    const int nl = 2 * nseq;
    const long nrows = (long)a.ny * a.nz;
    long row0;
    int k0, j0;
    if constexpr (NF > 0) {
        // tiles in (row tile, plane) order, plane fastest: the tile of the
        // same rows one plane up, whose rows of w (or p) this tile also
        // reads, is the next workgroup on the same XCD (an L2 hit)
        const int b = (int)xcd_remap(blockIdx.x, gridDim.x);
        const int jt = b / a.nz;
        k0 = b - jt * a.nz;
        j0 = jt * nl;
        row0 = (long)k0 * a.ny + j0;
    } else {
        row0 = xcd_remap(blockIdx.x, gridDim.x) * nl;
        k0 = (int)(row0 / a.ny);
        j0 = (int)(row0 - (long)k0 * a.ny);
    }
    const size_t base = (size_t)row0 * N;
    TO* twl = lds_twiddle_ptr<TO>();
    TwiddleRegs<TO, NTHR, (NF > 0 ? NF : 1)> twr;
    if constexpr (NF == 0) stage_twiddles<TO, NTHR>(twl, a.twc, a.tws, N);
    else twr.load(a.twc, a.tws);
    double* __restrict__ out_f = a.out_f;
    constexpr int PPW = NF > 0 ? NF / NTHR / 2 : 1;
    TO pw[PPW][4];   // fixed path: post-twiddles (cos, sin) of outputs i and i + 1
    double ss = 0.0, s1 = 0.0, s2 = 0.0, sp = 0.0;
    if constexpr (NF > 0) {
        static_assert(NF % NTHR == 0, "fixed x path: whole columns per thread");
        constexpr int CPR = NF / NTHR, NL = 2 * NSF;
        // rows per load batch (the residual stencil loads 8 values per cell:
        // two rows keep its registers within four waves per SIMD)
        constexpr bool RES = PRO == PRO_RESID || PRO == PRO_RESID_F;
        constexpr int RB0 = (RES || (PRO == PRO_DIV && sizeof(TO) == 4)) ? 2 : 4;
        constexpr int RB = (NL % RB0 == 0) ? RB0 : ((NL % 2 == 0) ? 2 : 1);
        // each thread owns the adjacent columns (2q, 2q + 1), q = tid + c NTHR
        constexpr int PPR = CPR / 2;
        static_assert(CPR % 2 == 0, "column pairs");
        PairNb cn[PPR];
        int lp0[PPR], lp1[PPR];
        // post-twiddles of the outputs this thread stores (m = i, i + 1),
        // loaded before the field rows
        // (unconditionally: the tables exist for both boundary kinds, and a
        // periodic line ignores them)
#pragma unroll
        for (int c = 0; c < PPR; ++c) {
            const int i = 2 * (threadIdx.x + c * NTHR);
            pw[c][0] = a.dctc[i];
            pw[c][1] = a.dcts[i];
            pw[c][2] = a.dctc[i + 1];
            pw[c][3] = a.dcts[i + 1];
        }
#pragma unroll
        for (int c = 0; c < PPR; ++c) {
            const int i = 2 * (threadIdx.x + c * NTHR);
            cn[c] = pair_nb(i, NF, a.bcx);
            lp0[c] = li(0, (a.bcx == FSEI_BC_WALL) ? mk_pos(i, NF) : i, SP);
            lp1[c] = li(0, (a.bcx == FSEI_BC_WALL) ? mk_pos(i + 1, NF) : i + 1, SP);
        }
        // residual prologue: the iterate's rows carried down the tile (rows
        // l - 1 and l in registers, row l + 1 loaded; the tile's first and
        // last rows take their outer neighbours from row_nb), so a row costs
        // 6 loads instead of 8; same arithmetic as x_prologue_pair
        double2 pprev[PPR], pcur[PPR];
        typename Vec2T<TI>::type vcur[PPR];
        if constexpr (PRO == PRO_DIV || PRO == PRO_DIV_ADJ) {
#pragma unroll
            for (int c = 0; c < PPR; ++c) vcur[c] = *reinterpret_cast<const typename Vec2T<TI>::type*>(a.v + base + cn[c].i);
        }
        if constexpr (RES) {
            const auto* __restrict__ pp = resid_iterate<PRO>(a) + base;
            const RowNb rn0 = row_nb(k0, j0, NF, a.ny, a.nz, a.bcy);
#pragma unroll
            for (int c = 0; c < PPR; ++c) {
                pcur[c] = pair_d(pp + cn[c].i);
                pprev[c] = pair_d(pp + rn0.ym + (long)cn[c].i);
            }
        }
#pragma unroll
        for (int l0 = 0; l0 < NL; l0 += RB) {
            TI val0[RB][PPR], val1[RB][PPR];
            if constexpr (RES) {
                // the host launches this path only when ny is a multiple of
                // the rows per tile, so all rows of a tile share plane k0
                const auto* __restrict__ pp = resid_iterate<PRO>(a) + base;
                double2 pn[RB][PPR], pzp[RB][PPR], pzm[RB][PPR], fc[RB][PPR];
                double pxm[RB][PPR], pxp[RB][PPR];
#pragma unroll
                for (int lr = 0; lr < RB; ++lr) {
                    const int l = l0 + lr;
                    const RowNb rn = row_nb(k0, j0 + l, NF, a.ny, a.nz, a.bcy);
                    const long ynext = (l + 1 < NL) ? (long)NF : rn.yp;
#pragma unroll
                    for (int c = 0; c < PPR; ++c) {
                        const long ro = (long)l * NF + cn[c].i;
                        pn[lr][c] = pair_d(pp + ro + ynext);
                        pzp[lr][c] = pair_d(pp + ro + rn.zp);
                        pzm[lr][c] = pair_d(pp + ro + rn.zm);
                        fc[lr][c] = *reinterpret_cast<const double2*>(a.f + base + ro);
                        pxm[lr][c] = (double)pp[(long)l * NF + cn[c].im];
                        pxp[lr][c] = (double)pp[(long)l * NF + cn[c].ip2];
                    }
                }
                const double zc = a.zc[k0], za = a.za[k0], mean = a.scal[0];
#pragma unroll
                for (int lr = 0; lr < RB; ++lr) {
                    const int l = l0 + lr;
                    const RowNb rn = row_nb(k0, j0 + l, NF, a.ny, a.nz, a.bcy);
#pragma unroll
                    for (int c = 0; c < PPR; ++c) {
                        const double2 pc = pcur[c], pym = pprev[c], pyp = pn[lr][c];
                        const double lx0 = (pc.y - pc.x) + (cn[c].him ? pxm[lr][c] - pc.x : 0.0);
                        const double lx1 = (cn[c].hip2 ? pxp[lr][c] - pc.y : 0.0) + (pc.x - pc.y);
                        const double ly0 = (rn.hyp ? pyp.x - pc.x : 0.0) + (rn.hym ? pym.x - pc.x : 0.0);
                        const double ly1 = (rn.hyp ? pyp.y - pc.y : 0.0) + (rn.hym ? pym.y - pc.y : 0.0);
                        const double lz0 = (rn.hzp ? zc * (pzp[lr][c].x - pc.x) : 0.0) +
                                           (rn.hzm ? za * (pzm[lr][c].x - pc.x) : 0.0);
                        const double lz1 = (rn.hzp ? zc * (pzp[lr][c].y - pc.y) : 0.0) +
                                           (rn.hzm ? za * (pzm[lr][c].y - pc.y) : 0.0);
                        val0[lr][c] = (TI)((fc[lr][c].x - mean) - (lx0 * a.idx2 + ly0 * a.idy2 + lz0));
                        val1[lr][c] = (TI)((fc[lr][c].y - mean) - (lx1 * a.idx2 + ly1 * a.idy2 + lz1));
                        sp += pc.x + pc.y;
                        pprev[c] = pc;
                        pcur[c] = pyp;
                    }
                }
            } else if constexpr (PRO == PRO_DIV || PRO == PRO_DIV_ADJ) {
                // divergence: v carried down the tile like the residual's
                // iterate (row l + 1 of v is row l's y+1 face), 5 loads per row
                using V = typename Vec2T<TI>::type;
                V uc[RB][PPR], vn[RB][PPR], wc[RB][PPR], wh[RB][PPR], gv[RB][PPR];
                TI uh[RB][PPR];
#pragma unroll
                for (int lr = 0; lr < RB; ++lr) {
                    const int l = l0 + lr;
                    const RowNb rn = row_nb(k0, j0 + l, NF, a.ny, a.nz, a.bcy);
                    const long ynext = (l + 1 < NL) ? (long)NF : rn.yp;
#pragma unroll
                    for (int c = 0; c < PPR; ++c) {
                        const size_t ro = base + (size_t)l * NF;
                        uc[lr][c] = *reinterpret_cast<const V*>(a.u + ro + cn[c].i);
                        uh[lr][c] = a.u[ro + cn[c].ip2];
                        vn[lr][c] = *reinterpret_cast<const V*>(a.v + (long)(ro + cn[c].i) + ynext);
                        wc[lr][c] = *reinterpret_cast<const V*>(a.w + ro + cn[c].i);
                        wh[lr][c] = *reinterpret_cast<const V*>(a.w + (long)(ro + cn[c].i) + rn.zp);
                        if constexpr (PRO == PRO_DIV_ADJ) {
                            if (a.gp) gv[lr][c] = *reinterpret_cast<const V*>(a.gp + ro + cn[c].i);
                        }
                    }
                }
                const TI zk = a.zeta[k0], ek = a.eta[k0], zero = (TI)0;
#pragma unroll
                for (int lr = 0; lr < RB; ++lr) {
                    const int l = l0 + lr;
                    const RowNb rn = row_nb(k0, j0 + l, NF, a.ny, a.nz, a.bcy);
#pragma unroll
                    for (int c = 0; c < PPR; ++c) {
                        const V vc = vcur[c], vh = vn[lr][c];
                        TI r0 = (uc[lr][c].y - (cn[c].him ? uc[lr][c].x : zero)) * a.idx +
                                ((rn.hyp ? vh.x : zero) - (rn.hym ? vc.x : zero)) * a.idy +
                                (zk * (rn.hzp ? wh[lr][c].x : zero) - ek * (rn.hzm ? wc[lr][c].x : zero));
                        TI r1 = ((cn[c].hip2 ? uh[lr][c] : zero) - uc[lr][c].y) * a.idx +
                                ((rn.hyp ? vh.y : zero) - (rn.hym ? vc.y : zero)) * a.idy +
                                (zk * (rn.hzp ? wh[lr][c].y : zero) - ek * (rn.hzm ? wc[lr][c].y : zero));
                        r0 *= a.alpha;
                        r1 *= a.alpha;
                        if constexpr (PRO == PRO_DIV_ADJ) {
                            if (a.gp) {
                                r0 += a.beta * gv[lr][c].x;
                                r1 += a.beta * gv[lr][c].y;
                            }
                        }
                        val0[lr][c] = r0;
                        val1[lr][c] = r1;
                        vcur[c] = vh;
                    }
                }
            } else {
#pragma unroll
                for (int lr = 0; lr < RB; ++lr) {
                    const int l = l0 + lr;
                    const RowNb rn = row_nb(k0, j0 + l, NF, a.ny, a.nz, a.bcy);
#pragma unroll
                    for (int c = 0; c < PPR; ++c)
                        x_prologue_pair<TI, TO, PRO>(a, base + (size_t)l * NF, k0, rn, cn[c], val0[lr][c],
                                                     val1[lr][c]);
                }
            }
            if (l0 == 0) twr.store(twl);
#pragma unroll
            for (int lr = 0; lr < RB; ++lr) {
                const int l = l0 + lr;
#pragma unroll
                for (int c = 0; c < PPR; ++c) {
                    const double v0 = (double)val0[lr][c], v1 = (double)val1[lr][c];
                    if (out_f) *reinterpret_cast<double2*>(out_f + base + (size_t)l * NF + cn[c].i) = make_double2(v0, v1);
                    ss += v0 * v0 + v1 * v1;
                    s1 += v0 + v1;
                    TO* dst = (l & 1) ? sim : sre;
                    dst[(l >> 1) * SP + lp0[c]] = (TO)val0[lr][c];
                    dst[(l >> 1) * SP + lp1[c]] = (TO)val1[lr][c];
                }
            }
        }
        if (a.dzw) s2 = a.dzw[k0] * (RES ? sp : s1);   // every row of the tile is in plane k0
    } else {
        const int total = nl * N;
        constexpr int PER = 2 * EMAX / NTHR;   // elements per thread, >= total / NTHR
        constexpr int BAT = (PER % 4 == 0) ? 4 : 1;
        for (int r0 = 0; r0 < PER; r0 += BAT) {
            TI val[BAT];
#pragma unroll
            for (int r = 0; r < BAT; ++r) {
                const int e = threadIdx.x + (r0 + r) * NTHR;
                val[r] = (TI)0;
                if (e < total) {
                    const int l = e / N;
                    const int i = e - l * N;
                    if (row0 + l < nrows) {
                        int k, j;
                        row_kj(k0, j0, l, a.ny, k, j);
                        val[r] = x_prologue<TI, TO, PRO>(a, base, k, j, i, e, N);
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < BAT; ++r) {
                const int e = threadIdx.x + (r0 + r) * NTHR;
                if (e < total) {
                    const int l = e / N;
                    const int i = e - l * N;
                    if (row0 + l < nrows) {
                        if (out_f) out_f[base + e] = (double)val[r];
                        ss += (double)val[r] * (double)val[r];
                        s1 += (double)val[r];
                        if (a.dzw) {
                            int k, j;
                            row_kj(k0, j0, l, a.ny, k, j);
                            constexpr bool RES = PRO == PRO_RESID || PRO == PRO_RESID_F;
                            s2 += a.dzw[k] * (RES ? (double)resid_iterate<PRO>(a)[base + e] : (double)val[r]);
                        }
                    }
                    const int n = (a.bcx == FSEI_BC_WALL) ? mk_pos(i, N) : i;
                    if (l & 1) sim[li(l >> 1, n, SP)] = (TO)val[r];
                    else sre[li(l >> 1, n, SP)] = (TO)val[r];
                }
            }
        }
    }
    if (a.partials) {
        block_sum3<NTHR>(ss, s1, s2, sred);
        if (threadIdx.x == 0) {
            a.partials[3 * blockIdx.x] = ss;
            a.partials[3 * blockIdx.x + 1] = s1;
            a.partials[3 * blockIdx.x + 2] = s2;
        }
    } else {
        __syncthreads();
    }
    if (a.out == nullptr) return;   // norm-only pass (uniform over the block)
    fft_lds<TO, EMAX, NTHR, -1, NF>(sre, sim, N, nseq, a.fp, twl, twl + N);
    TO* __restrict__ out = a.out + base;
    if constexpr (NF > 0) {
        // outputs m, m + 1 (m even) of every line pair, stored as pairs
        using VO = typename Vec2T<TO>::type;
        constexpr int PPR = NF / NTHR / 2;
#pragma unroll
        for (int c = 0; c < PPR; ++c) {
            const int m0 = 2 * (threadIdx.x + c * NTHR), m1 = m0 + 1;
            const int mm0 = (m0 == 0) ? 0 : NF - m0, mm1 = NF - m1;
            const int l0 = li(0, m0, SP), lm0 = li(0, mm0, SP), l1 = li(0, m1, SP), lm1 = li(0, mm1, SP);
            const bool lo0 = 2 * m0 <= NF, lo1 = 2 * m1 <= NF;
            const TO wr0 = pw[c][0], wi0 = -pw[c][1], wr1 = pw[c][2], wi1 = -pw[c][3];
#pragma unroll
            for (int s = 0; s < NSF; ++s) {
                VO xa, xb;
                post_fwd_v<TO>(a.bcx, lo0, sre[s * SP + l0], sim[s * SP + l0], sre[s * SP + lm0], sim[s * SP + lm0],
                               wr0, wi0, xa.x, xb.x);
                post_fwd_v<TO>(a.bcx, lo1, sre[s * SP + l1], sim[s * SP + l1], sre[s * SP + lm1], sim[s * SP + lm1],
                               wr1, wi1, xa.y, xb.y);
                *reinterpret_cast<VO*>(out + (2 * s) * NF + m0) = xa;
                *reinterpret_cast<VO*>(out + (2 * s + 1) * NF + m0) = xb;
            }
        }
    } else {
        constexpr int PST = EMAX / NTHR;
#pragma unroll
        for (int r = 0; r < PST; ++r) {
            const int e = threadIdx.x + r * NTHR;
            if (e < nseq * N) {
                const int s = e / N;
                const int m = e - s * N;
                TO xa, xb;
                post_fwd<TO>(sre, sim, s, SP, N, m, a.bcx, a.dctc, a.dcts, xa, xb);
                if (row0 + 2 * s < nrows) out[2 * s * N + m] = xa;
                if (row0 + 2 * s + 1 < nrows) out[(2 * s + 1) * N + m] = xb;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// x inverse: unnormalised inverse x transform of row pairs; writes (STORE)
// or adds (ACC) the result into the output field
// ---------------------------------------------------------------------------
// STORE: out = result; ACC: out += result; ADDF: out = add32 + result;
// ACC_KEEP: out += result and the result is also written back over the input
enum { EPI_STORE = 0, EPI_ACC = 1, EPI_ADDF = 2, EPI_ACC_KEEP = 3 };

template <typename T, typename TP>
struct XInvArgs {
    int nx, ny, nz, bcx, nseq;
    FftPlan fp;
    const T* in;
    TP* out;
    const float* add32;   // EPI_ADDF: FP32 field added to the result
    T* keep;              // EPI_ACC_KEEP: receives the result (the input field itself)
    const double* vsum;   // ACC / ADDF: if set, vsum[0] * vscale is subtracted from
    double vscale;        //   every output (the V-mean of the previous iterate)
    const T* twc;
    const T* tws;
    const T* dctc;
    const T* dcts;
};

template <typename T, typename TP, int EPI, int EMAX, int NTHR, int NF>
__global__ __launch_bounds__(NTHR) void k_xinv(XInvArgs<T, TP> a) {
    __shared__ T sre[lds_elems(EMAX)];
    __shared__ T sim[lds_elems(EMAX)];
    constexpr int NSF = NF > 0 ? tile_nseq(EMAX, NF) : 0;
    const int N = NF > 0 ? NF : a.nx;
    const int SP = seq_stride(N);
    const int nseq = NF > 0 ? NSF : a.nseq;
    const int nl = 2 * nseq;
    const long row0 = xcd_remap(blockIdx.x, gridDim.x) * nl;
    const long nrows = (long)a.ny * a.nz;
    const size_t base = (size_t)row0 * N;
    const T* in = a.in + base;   // not restrict: ACC_KEEP writes this field back (after every read of it)
    T* twl = lds_twiddle_ptr<T>();
    TwiddleRegs<T, NTHR, (NF > 0 ? NF : 1)> twr;
    if constexpr (NF == 0) stage_twiddles<T, NTHR>(twl, a.twc, a.tws, N);
    else twr.load(a.twc, a.tws);
    if constexpr (NF > 0) {
        static_assert(NF % NTHR == 0, "fixed x path: whole columns per thread");
        constexpr int CPR = NF / NTHR;
        static_assert(CPR % 2 == 0, "paired columns");
        // each thread loads columns m < NF/2 and its partner NF - m once and
        // forms both pre-twiddled values (m = 0 pairs with NF/2; both of
        // those use only their own column)
#pragma unroll
        for (int c = 0; c < CPR / 2; ++c) {
            const int m = threadIdx.x + c * NTHR;
            const int nm = (m == 0) ? NF / 2 : NF - m;
            const int lm = li(0, m, SP), lnm = li(0, nm, SP);
            // pre-twiddles, loaded before the rows and unconditionally (a
            // periodic line ignores them); cos/sin(pi m / 2NF) at NF - m
            // are sin/cos at m
            T cm = a.dctc[m], sm = a.dcts[m], c0 = a.dctc[NF / 2], s0 = a.dcts[NF / 2];
            T xam[NSF], xanm[NSF], xbm[NSF], xbnm[NSF];
#pragma unroll
            for (int s = 0; s < NSF; ++s) {
                xam[s] = in[(2 * s) * NF + m];
                xanm[s] = in[(2 * s) * NF + nm];
                xbm[s] = in[(2 * s + 1) * NF + m];
                xbnm[s] = in[(2 * s + 1) * NF + nm];
            }
            // (not used before the rows are requested)
            asm volatile("" : "+v"(cm), "+v"(sm), "+v"(c0), "+v"(s0));
            const T cn = (m == 0) ? c0 : sm, sn = (m == 0) ? s0 : cm;
            if (c == 0) twr.store(twl);
#pragma unroll
            for (int s = 0; s < NSF; ++s) {
                const T pa = (m == 0) ? xanm[s] : xam[s], pb = (m == 0) ? xbnm[s] : xbm[s];
                T zr, zi;
                pre_inv_cs<T>(NF, m, a.bcx, xam[s], xanm[s], xbm[s], xbnm[s], cm, sm, zr, zi);
                sre[s * SP + lm] = zr;
                sim[s * SP + lm] = zi;
                pre_inv_cs<T>(NF, nm, a.bcx, xanm[s], pa, xbnm[s], pb, cn, sn, zr, zi);
                sre[s * SP + lnm] = zr;
                sim[s * SP + lnm] = zi;
            }
        }
    } else {
        constexpr int PLD = EMAX / NTHR;
#pragma unroll
        for (int r = 0; r < PLD; ++r) {
            const int e = threadIdx.x + r * NTHR;
            if (e < nseq * N) {
                const int s = e / N;
                const int m = e - s * N;
                const int nm = (m == 0) ? 0 : N - m;
                T xam = 0, xanm = 0, xbm = 0, xbnm = 0;
                if (row0 + 2 * s < nrows) {
                    xam = in[2 * s * N + m];
                    xanm = in[2 * s * N + nm];
                }
                if (row0 + 2 * s + 1 < nrows) {
                    xbm = in[(2 * s + 1) * N + m];
                    xbnm = in[(2 * s + 1) * N + nm];
                }
                T zr, zi;
                pre_inv<T>(N, m, a.bcx, xam, xanm, xbm, xbnm, a.dctc, a.dcts, zr, zi);
                sre[li(s, m, SP)] = zr;
                sim[li(s, m, SP)] = zi;
            }
        }
    }
    TP* __restrict__ out = a.out + base;
    // fixed path, accumulating epilogues: the values the result is added to
    // (the iterate, or the FP32 field) are loaded before the transform and
    // arrive while it runs
    constexpr bool ACCF = NF > 0 && (EPI == EPI_ACC || EPI == EPI_ADDF || EPI == EPI_ACC_KEEP);
    constexpr int NLA = ACCF ? 2 * NSF : 1, PPA = ACCF ? NF / NTHR / 2 : 1;
    using VPA = typename Vec2T<TP>::type;
    VPA old[NLA][PPA];
    if constexpr (ACCF) {
        const float* __restrict__ add = (EPI == EPI_ADDF) ? a.add32 + base : nullptr;
#pragma unroll
        for (int l = 0; l < NLA; ++l)
#pragma unroll
            for (int c = 0; c < PPA; ++c) {
                const int o = l * NF + 2 * (threadIdx.x + c * NTHR);
                if constexpr (EPI == EPI_ADDF) {
                    const float2 q = *reinterpret_cast<const float2*>(add + o);
                    old[l][c].x = (TP)q.x;
                    old[l][c].y = (TP)q.y;
                } else {
                    old[l][c] = *reinterpret_cast<const VPA*>(out + o);
                }
            }
    }
    __syncthreads();
    fft_lds<T, EMAX, NTHR, 1, NF>(sre, sim, N, nseq, a.fp, twl, twl + N);
    if constexpr (NF > 0) {
        // outputs i, i + 1 (i even) of every line, read and written as pairs
        using VT = typename Vec2T<T>::type;
        using VP = typename Vec2T<TP>::type;
        constexpr int PPR = NF / NTHR / 2, NL = 2 * NSF;
        static_assert(NF % (2 * NTHR) == 0, "column pairs");
        int ln0[PPR], ln1[PPR];
#pragma unroll
        for (int c = 0; c < PPR; ++c) {
            const int i = 2 * (threadIdx.x + c * NTHR);
            ln0[c] = li(0, (a.bcx == FSEI_BC_WALL) ? mk_pos(i, NF) : i, SP);
            ln1[c] = li(0, (a.bcx == FSEI_BC_WALL) ? mk_pos(i + 1, NF) : i + 1, SP);
        }
        if constexpr (ACCF) {
            static_assert(NLA == NL && PPA == PPR, "prefetched epilogue values");
            const TP msub = a.vsum ? (TP)(a.vsum[0] * a.vscale) : (TP)0;
#pragma unroll
            for (int l = 0; l < NL; ++l)
#pragma unroll
                for (int c = 0; c < PPR; ++c) {
                    old[l][c].x -= msub;
                    old[l][c].y -= msub;
                }
#pragma unroll
            for (int l = 0; l < NL; ++l)
#pragma unroll
                for (int c = 0; c < PPR; ++c) {
                    const int o = l * NF + 2 * (threadIdx.x + c * NTHR);
                    const T* src = (l & 1) ? sim : sre;
                    VT val;
                    val.x = src[(l >> 1) * SP + ln0[c]];
                    val.y = src[(l >> 1) * SP + ln1[c]];
                    VP r;
                    r.x = old[l][c].x + (TP)val.x;
                    r.y = old[l][c].y + (TP)val.y;
                    *reinterpret_cast<VP*>(out + o) = r;
                    if constexpr (EPI == EPI_ACC_KEEP) *reinterpret_cast<VT*>(a.keep + base + o) = val;
                }
        } else {
#pragma unroll
            for (int l = 0; l < NL; ++l)
#pragma unroll
                for (int c = 0; c < PPR; ++c) {
                    const int o = l * NF + 2 * (threadIdx.x + c * NTHR);
                    const T* src = (l & 1) ? sim : sre;
                    VP r;
                    r.x = (TP)src[(l >> 1) * SP + ln0[c]];
                    r.y = (TP)src[(l >> 1) * SP + ln1[c]];
                    *reinterpret_cast<VP*>(out + o) = r;
                }
        }
    } else {
        constexpr int PST = 2 * EMAX / NTHR;
        const TP msub = (EPI != EPI_STORE && a.vsum) ? (TP)(a.vsum[0] * a.vscale) : (TP)0;
#pragma unroll
        for (int r = 0; r < PST; ++r) {
            const int e = threadIdx.x + r * NTHR;
            if (e < nl * N) {
                const int l = e / N;
                const int i = e - l * N;
                if (row0 + l < nrows) {
                    const int n = (a.bcx == FSEI_BC_WALL) ? mk_pos(i, N) : i;
                    const T val = (l & 1) ? sim[li(l >> 1, n, SP)] : sre[li(l >> 1, n, SP)];
                    if constexpr (EPI == EPI_ACC) out[e] = (out[e] - msub) + (TP)val;
                    else if constexpr (EPI == EPI_ADDF) out[e] = ((TP)a.add32[base + e] - msub) + (TP)val;
                    else if constexpr (EPI == EPI_ACC_KEEP) {
                        out[e] = (out[e] - msub) + (TP)val;
                        a.keep[base + e] = val;
                    } else out[e] = (TP)val;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// x inverse fused with the gradient correction (paper, Sec. 2.1, eq.
// NSdiscr0: the pressure term -dt grad p^{n+1} applied to the provisional
// velocity), FP64, compile-time length NF, one column pair per thread:
//     p = inverse x transform of the y-inverted field,
//     u += cx (p_i - p_{i-1}),  v += cy (p_j - p_{j-1}),
//     w += sw (bk_k p_k - gk_k p_{k-1}),
// on active faces (wall faces written 0), p written once (optional) and never
// re-read.  A workgroup owns GR = 8 rows j0..j0+7 over a chunk of planes and
// marches up in z.  Each step inverts the 8 rows plus row j0-1 (whose p the v
// update of row j0 needs) of one plane: 9 real rows as 5 complex sequences,
// the last paired with a zero row.  The own rows' p of the previous plane
// stay in registers for the w update; the chunk's first step only produces
// them (it inverts the plane below the chunk).
// ---------------------------------------------------------------------------
struct XInvGradArgs {
    int ny, nz, bcx, bcy, kc;   // kc: planes per chunk
    const double* in;           // y-inverted field (transform space in x)
    double* p;                  // pressure out, or null
    double* u;
    double* v;
    double* w;
    double cx, cy, sw;
    const double* bk;
    const double* gk;
    const double* twc;
    const double* tws;
    const double* dctc;
    const double* dcts;
};

// two adjacent doubles as one non-temporal 16-byte store
__device__ __forceinline__ void nt_store2(double* q, double2 v) {
    __builtin_nontemporal_store(v.x, q);
    __builtin_nontemporal_store(v.y, q + 1);
}

constexpr int kXgRows = 8;    // own rows per workgroup
constexpr int kXgSeq = 5;     // complex sequences per step (8 rows + halo + zero row)

// Threads: one per radix-8 butterfly of a stage (5 NF / 8); the first NF / 2
// also own one column (pair) each in the load and gradient phases.
template <int NF>
constexpr int xg_threads() { return kXgSeq * NF / 8; }

template <int NF>
__global__ __launch_bounds__(xg_threads<NF>()) void k_xinv_grad(XInvGradArgs a) {
    constexpr int NTHR = xg_threads<NF>();
    constexpr int GR = kXgRows, NSQ = kXgSeq, EMAX = NSQ * NF;
    static_assert(NTHR >= NF / 2, "a column pair per thread");
    constexpr int SP = seq_stride(NF);
    constexpr int GB = 4;   // rows per batch of the gradient phase
    static_assert(NSQ * SP <= lds_elems(EMAX), "tile fits");
    static_assert(2 * NSQ == GR + 2, "halo row + own rows + one zero row");
    static_assert(GR % GB == 0, "whole batches");
    __shared__ double sre[lds_elems(EMAX)];
    __shared__ double sim[lds_elems(EMAX)];
    const int ny = a.ny, nz = a.nz;
    const int ntj = ny / GR;
    const int b = (int)xcd_remap(blockIdx.x, gridDim.x);
    const int chunk = b / ntj;
    const int jt = b - chunk * ntj;
    const int j0 = jt * GR;
    const int kb = chunk * a.kc;
    const int ke = (kb + a.kc < nz) ? kb + a.kc : nz;
    const int jh = (j0 > 0) ? j0 - 1 : ny - 1;   // halo row (wrapped; unused for a y wall at j0 = 0)
    const bool wallx = a.bcx == FSEI_BC_WALL, wally = a.bcy == FSEI_BC_WALL;
    double* twl = lds_twiddles<double, NTHR>(a.twc, a.tws, NF);
    const bool colt = threadIdx.x < NF / 2;   // owns a column (pair)
    // pre-processing: column m and its partner nm of every row
    const int m = colt ? threadIdx.x : 0;
    const int nm = (m == 0) ? NF / 2 : NF - m;
    const int lm = li(0, m, SP), lnm = li(0, nm, SP);
    double cm = 1.0, sm = 0.0, cn = 1.0, sn = 0.0;
    if (wallx) {
        cm = a.dctc[m];
        sm = a.dcts[m];
        cn = (m == 0) ? a.dctc[NF / 2] : sm;
        sn = (m == 0) ? a.dcts[NF / 2] : cm;
    }
    // gradient: this thread's column pair (i, i + 1) and the x neighbour i - 1
    const int i = 2 * m;
    const int ixm = (i > 0) ? i - 1 : NF - 1;
    const int q0 = li(0, wallx ? mk_pos(i, NF) : i, SP);
    const int q1 = li(0, wallx ? mk_pos(i + 1, NF) : i + 1, SP);
    const int qm = li(0, wallx ? mk_pos(ixm, NF) : ixm, SP);
    const size_t plane = (size_t)NF * ny;
    // input rows of one step: tile row r = 0 is the halo row, r = 1..8 the
    // own rows, r = 9 zero; sequence s pairs rows 2s and 2s + 1
    double xa[NSQ][2], xb[NSQ][2];
    auto load_in = [&](int k) {
        const double* __restrict__ in = a.in + (size_t)k * plane;
#pragma unroll
        for (int s = 0; s < NSQ; ++s) {
            const int ra = 2 * s, rb = 2 * s + 1;
            const double* pa = in + (size_t)((ra == 0) ? jh : j0 + ra - 1) * NF;
            xa[s][0] = pa[m];
            xa[s][1] = pa[nm];
            if (rb <= GR) {
                const double* pb = in + (size_t)(j0 + rb - 1) * NF;
                xb[s][0] = pb[m];
                xb[s][1] = pb[nm];
            } else {
                xb[s][0] = 0.0;
                xb[s][1] = 0.0;
            }
        }
    };
    auto pv = [&](int r, int q) -> double { return ((r & 1) ? sim : sre)[(r >> 1) * SP + q]; };
    double2 prev[GR];
#pragma unroll
    for (int l = 0; l < GR; ++l) prev[l] = make_double2(0.0, 0.0);
    int k = (kb > 0) ? kb - 1 : 0;
    for (; k < ke; ++k) {
        if (colt) load_in(k);
#pragma unroll
        for (int s = 0; s < NSQ && colt; ++s) {
            const double pa = (m == 0) ? xa[s][1] : xa[s][0], pb = (m == 0) ? xb[s][1] : xb[s][0];
            double zr, zi;
            pre_inv_cs<double>(NF, m, a.bcx, xa[s][0], xa[s][1], xb[s][0], xb[s][1], cm, sm, zr, zi);
            sre[s * SP + lm] = zr;
            sim[s * SP + lm] = zi;
            pre_inv_cs<double>(NF, nm, a.bcx, xa[s][1], pa, xb[s][1], pb, cn, sn, zr, zi);
            sre[s * SP + lnm] = zr;
            sim[s * SP + lnm] = zi;
        }
        __syncthreads();
        fft_lds<double, EMAX, NTHR, 1, NF>(sre, sim, NF, NSQ, FftPlan{}, twl, twl + NF);
        // the next step's input is in flight during this step's gradient
        double2 pym = make_double2(pv(0, q0), pv(0, q1));
        if (!colt) {
        } else if (k >= kb) {   // not the chunk's first (halo) plane
            const double bkk = a.bk[k], gkk = a.gk[k];
            const size_t ro = (size_t)k * plane + (size_t)j0 * NF + i;
#pragma unroll
            for (int l0 = 0; l0 < GR; l0 += GB) {
                double2 uo[GB], vo[GB], wo[GB];
#pragma unroll
                for (int t = 0; t < GB; ++t) {
                    const size_t o = ro + (size_t)(l0 + t) * NF;
                    uo[t] = *reinterpret_cast<const double2*>(a.u + o);
                    vo[t] = *reinterpret_cast<const double2*>(a.v + o);
                    wo[t] = *reinterpret_cast<const double2*>(a.w + o);
                }
#pragma unroll
                for (int t = 0; t < GB; ++t) {
                    const int l = l0 + t, r = l + 1;
                    const double2 pc = make_double2(pv(r, q0), pv(r, q1));
                    const double pxm = pv(r, qm);
                    const int j = j0 + l;
                    double2 un, vn, wn;
                    un.x = (wallx && i == 0) ? 0.0 : uo[t].x + a.cx * (pc.x - pxm);
                    un.y = uo[t].y + a.cx * (pc.y - pc.x);
                    const bool v0 = wally && j == 0;
                    vn.x = v0 ? 0.0 : vo[t].x + a.cy * (pc.x - pym.x);
                    vn.y = v0 ? 0.0 : vo[t].y + a.cy * (pc.y - pym.y);
                    wn.x = (k == 0) ? 0.0 : wo[t].x + a.sw * (bkk * pc.x - gkk * prev[l].x);
                    wn.y = (k == 0) ? 0.0 : wo[t].y + a.sw * (bkk * pc.y - gkk * prev[l].y);
                    // non-temporal: nothing here is read again soon
                    const size_t o = ro + (size_t)l * NF;
                    nt_store2(a.u + o, un);
                    nt_store2(a.v + o, vn);
                    nt_store2(a.w + o, wn);
                    if (a.p) nt_store2(a.p + o, pc);
                    prev[l] = pc;
                    pym = pc;
                }
                // keep the next batch's loads after this batch's stores
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
#pragma unroll
            for (int l = 0; l < GR; ++l) prev[l] = make_double2(pv(l + 1, q0), pv(l + 1, q1));
        }
        __syncthreads();   // the next step overwrites the tile
    }
}

// ---------------------------------------------------------------------------
// The first correction of the FP32 + FP64 refinement fused with the gradient
// correction and the convergence check (one pass instead of the x inverse
// with the ADDF epilogue followed by the gradient + residual kernel):
//     delta = FP32 inverse x transform of the y-inverted correction,
//     p = (p32 - m) + delta        in FP64 (m: V-mean of the first solve),
//     u += cx (p_i - p_{i-1}),  v += cy (p_j - p_{j-1}),
//     w += sw (bk_k p_k - gk_k p_{k-1})        (wall faces written 0),
//     r = (f - mean) - L p,  per-workgroup partials of sum r^2 and sum r,
// p written once.  The marching of k_xinv_grad, with 10 rows per plane
// (halo rows j0-1 and j0+8, both needed by the Laplacian) as 5 complex FP32
// sequences.  The residual of plane k needs p of plane k+1: its part
// without that term is kept in registers and completed one step later (the
// chunk's march takes one plane beyond its end when there is one).
// Every p is formed from p32 and delta exactly as the ADDF epilogue forms it.
// ---------------------------------------------------------------------------
struct XInvGradResArgs {
    int ny, nz, bcx, bcy, kc;
    const float* in;        // y-inverted correction (transform space in x), FP32
    const float* p32;       // first solve
    const double* vsum;     // vsum[0] * vscale is subtracted from p32
    double vscale;
    double* p;              // pressure out (FP64)
    double* u;
    double* v;
    double* w;
    double cx, cy, sw;
    const double* bk;
    const double* gk;
    const double* f;        // FP64 right-hand side
    double idx2, idy2;
    const double* za;
    const double* zc;
    const double* scal;     // scal[0] = removed mean of f
    double* partials;       // per workgroup: sum r^2, sum r, 0
    const float* twc;
    const float* tws;
    const float* dctc;
    const float* dcts;
};

// threads of k_xinv_grad_resid: one per column pair at 512 (two workgroups
// per CU fit the registers), one per radix-8 butterfly at 768
template <int NF>
constexpr int xgr_threads() { return NF == 512 ? NF / 2 : xg_threads<NF>(); }

template <int NF>
__global__ __launch_bounds__(xgr_threads<NF>()) void k_xinv_grad_resid(XInvGradResArgs a) {
    constexpr int NTHR = xgr_threads<NF>();
    constexpr int GR = kXgRows, NSQ = kXgSeq, EMAX = NSQ * NF;
    static_assert(NTHR >= NF / 2, "a column pair per thread");
    constexpr int SP = seq_stride(NF);
    constexpr int GB = 2;   // rows per batch of the gradient phase
    static_assert(NSQ * SP <= lds_elems(EMAX), "tile fits");
    static_assert(2 * NSQ == GR + 2, "two halo rows + own rows");
    static_assert(GR % GB == 0, "whole batches");
    static_assert(NF / 2 <= 64 * (NTHR / 64), "the column-owning threads are in the waves block_sum3 adds");
    __shared__ float sre[lds_elems(EMAX)];
    __shared__ float sim[lds_elems(EMAX)];
    __shared__ double sred[3 * (NTHR / 64 + 1)];
    const int ny = a.ny, nz = a.nz;
    const int ntj = ny / GR;
    const int b = (int)xcd_remap(blockIdx.x, gridDim.x);
    const int chunk = b / ntj;
    const int jt = b - chunk * ntj;
    const int j0 = jt * GR;
    const int kb = chunk * a.kc;
    const int ke = (kb + a.kc < nz) ? kb + a.kc : nz;
    const int kend = (ke < nz) ? ke + 1 : ke;   // one plane beyond the chunk for its last residual
    const int jh = (j0 > 0) ? j0 - 1 : ny - 1;            // halo rows (wrapped; a y wall never uses them)
    const int jn = (j0 + GR < ny) ? j0 + GR : 0;
    const bool wallx = a.bcx == FSEI_BC_WALL, wally = a.bcy == FSEI_BC_WALL;
    float* twl = lds_twiddles<float, NTHR>(a.twc, a.tws, NF);
    const bool colt = threadIdx.x < NF / 2;   // owns a column (pair)
    const int m = colt ? threadIdx.x : 0;
    const int nm = (m == 0) ? NF / 2 : NF - m;
    const int lm = li(0, m, SP), lnm = li(0, nm, SP);
    float cm = 1.0f, sm = 0.0f, cn = 1.0f, sn = 0.0f;
    if (wallx) {
        cm = a.dctc[m];
        sm = a.dcts[m];
        cn = (m == 0) ? a.dctc[NF / 2] : sm;
        sn = (m == 0) ? a.dcts[NF / 2] : cm;
    }
    // this thread's column pair (i, i + 1) and its x neighbours i - 1, i + 2
    const int i = 2 * m;
    const int ixm = (i > 0) ? i - 1 : NF - 1;
    const int ixp = (i + 2 < NF) ? i + 2 : 0;
    const bool perx = !wallx, pery = !wally;
    const bool him = (i > 0) || perx, hip = (i + 2 < NF) || perx;
    const int q0 = li(0, wallx ? mk_pos(i, NF) : i, SP);
    const int q1 = li(0, wallx ? mk_pos(i + 1, NF) : i + 1, SP);
    const int qm = li(0, wallx ? mk_pos(ixm, NF) : ixm, SP);
    const int qp = li(0, wallx ? mk_pos(ixp, NF) : ixp, SP);
    const size_t plane = (size_t)NF * ny;
    const double msub = a.vsum ? a.vsum[0] * a.vscale : 0.0;
    const double mean = a.scal[0];
    auto rowj = [&](int r) { return (r == 0) ? jh : ((r <= GR) ? j0 + r - 1 : jn); };
    // step input: the correction's rows (tile row r = 0: row j0 - 1, 1..8:
    // own rows, 9: row j0 + 8; sequence s pairs rows 2s and 2s + 1)
    float xa[NSQ][2], xb[NSQ][2];
    auto load_in = [&](int k) {
        const float* __restrict__ in = a.in + (size_t)k * plane;
#pragma unroll
        for (int s = 0; s < NSQ; ++s) {
            const float* pa = in + (size_t)rowj(2 * s) * NF;
            const float* pb = in + (size_t)rowj(2 * s + 1) * NF;
            xa[s][0] = pa[m];
            xa[s][1] = pa[nm];
            xb[s][0] = pb[m];
            xb[s][1] = pb[nm];
        }
    };
    auto dl = [&](int r, int q) -> double { return (double)((r & 1) ? sim : sre)[(r >> 1) * SP + q]; };
    // p of tile row r at the thread's pair, from that row's p32 pair: (p32 - m) + delta, in FP64
    auto pair_p = [&](int r, float2 q) {
        return make_double2(((double)q.x - msub) + dl(r, q0), ((double)q.y - msub) + dl(r, q1));
    };
    double2 prev[GR];    // p of the plane below, own rows
    double2 rpart[GR];   // residual of the plane below without its z+1 term
#pragma unroll
    for (int l = 0; l < GR; ++l) {
        prev[l] = make_double2(0.0, 0.0);
        rpart[l] = make_double2(0.0, 0.0);
    }
    double ss = 0.0, s1 = 0.0;
    int k = (kb > 0) ? kb - 1 : 0;
    for (; k < kend; ++k) {
        if (colt) load_in(k);
#pragma unroll
        for (int s = 0; s < NSQ && colt; ++s) {
            const float pa = (m == 0) ? xa[s][1] : xa[s][0], pb = (m == 0) ? xb[s][1] : xb[s][0];
            float zr, zi;
            pre_inv_cs<float>(NF, m, a.bcx, xa[s][0], xa[s][1], xb[s][0], xb[s][1], cm, sm, zr, zi);
            sre[s * SP + lm] = zr;
            sim[s * SP + lm] = zi;
            pre_inv_cs<float>(NF, nm, a.bcx, xa[s][1], pa, xb[s][1], pb, cn, sn, zr, zi);
            sre[s * SP + lnm] = zr;
            sim[s * SP + lnm] = zi;
        }
        __syncthreads();
        fft_lds<float, EMAX, NTHR, 1, NF>(sre, sim, NF, NSQ, FftPlan{}, twl, twl + NF);
        // uniform over the workgroup: this plane's own rows get the gradient
        // (grad), complete the residual of the plane below (lag), or only
        // provide p for the next plane (the chunk's halo plane)
        const bool grad = k >= kb && k < ke;
        const bool lag = k - 1 >= kb && k - 1 < ke;
        if (colt) {
            const float* __restrict__ p3 = a.p32 + (size_t)k * plane + i;
            const size_t ro = (size_t)k * plane + (size_t)j0 * NF + i;
            const double bkk = a.bk[k], gkk = a.gk[k];
            const double czm = (k > 0) ? a.za[k] : 0.0;
            const double czl = (k > 0) ? a.zc[k - 1] : 0.0;   // z+1 coefficient of the plane below
            const bool hzm = k > 0, hzp = k + 1 < nz;
            double2 pym = make_double2(0.0, 0.0);
            if (grad) pym = pair_p(0, *reinterpret_cast<const float2*>(p3 + (size_t)jh * NF));
#pragma unroll
            for (int l0 = 0; l0 < GR; l0 += GB) {
                // p32 of tile rows l0+1 .. l0+GB+1 (the last one is the next
                // batch's first row, needed here for the y Laplacian)
                float2 q32[GB + 1];
                float qxm[GB], qxp[GB];
                double2 uo[GB], vo[GB], wo[GB], fo[GB];
#pragma unroll
                for (int t = 0; t <= GB; ++t) {
                    const int r = l0 + t + 1;
                    if (t < GB || grad) q32[t] = *reinterpret_cast<const float2*>(p3 + (size_t)rowj(r) * NF);
                }
                if (grad) {
#pragma unroll
                    for (int t = 0; t < GB; ++t) {
                        const size_t o = ro + (size_t)(l0 + t) * NF;
                        const float* pr = a.p32 + (o - i);
                        qxm[t] = pr[ixm];
                        qxp[t] = pr[ixp];
                        uo[t] = *reinterpret_cast<const double2*>(a.u + o);
                        vo[t] = *reinterpret_cast<const double2*>(a.v + o);
                        wo[t] = *reinterpret_cast<const double2*>(a.w + o);
                        fo[t] = *reinterpret_cast<const double2*>(a.f + o);
                    }
                }
#pragma unroll
                for (int t = 0; t < GB; ++t) {
                    const int l = l0 + t, r = l + 1;
                    const int j = j0 + l;
                    const double2 pc = pair_p(r, q32[t]);
                    if (lag) {   // the residual of the plane below, completed with this plane's p
                        const double r0 = rpart[l].x - czl * (pc.x - prev[l].x);
                        const double r1 = rpart[l].y - czl * (pc.y - prev[l].y);
                        ss += r0 * r0 + r1 * r1;
                        s1 += r0 + r1;
                    }
                    if (grad) {
                        const double2 pyp = pair_p(r + 1, q32[t + 1]);
                        const double pxm = ((double)qxm[t] - msub) + dl(r, qm);
                        const double pxp = ((double)qxp[t] - msub) + dl(r, qp);
                        // gradient correction
                        double2 un, vn, wn;
                        un.x = (wallx && i == 0) ? 0.0 : uo[t].x + a.cx * (pc.x - pxm);
                        un.y = uo[t].y + a.cx * (pc.y - pc.x);
                        const bool v0 = wally && j == 0;
                        vn.x = v0 ? 0.0 : vo[t].x + a.cy * (pc.x - pym.x);
                        vn.y = v0 ? 0.0 : vo[t].y + a.cy * (pc.y - pym.y);
                        wn.x = (k == 0) ? 0.0 : wo[t].x + a.sw * (bkk * pc.x - gkk * prev[l].x);
                        wn.y = (k == 0) ? 0.0 : wo[t].y + a.sw * (bkk * pc.y - gkk * prev[l].y);
                        // residual without the z+1 term
                        const bool hym = (j > 0) || pery, hyp = (j + 1 < ny) || pery;
                        const double lx0 = (pc.y - pc.x) + (him ? pxm - pc.x : 0.0);
                        const double lx1 = (hip ? pxp - pc.y : 0.0) + (pc.x - pc.y);
                        const double ly0 = (hyp ? pyp.x - pc.x : 0.0) + (hym ? pym.x - pc.x : 0.0);
                        const double ly1 = (hyp ? pyp.y - pc.y : 0.0) + (hym ? pym.y - pc.y : 0.0);
                        const double lz0 = hzm ? czm * (prev[l].x - pc.x) : 0.0;
                        const double lz1 = hzm ? czm * (prev[l].y - pc.y) : 0.0;
                        const double r0 = (fo[t].x - mean) - (lx0 * a.idx2 + ly0 * a.idy2 + lz0);
                        const double r1 = (fo[t].y - mean) - (lx1 * a.idx2 + ly1 * a.idy2 + lz1);
                        if (hzp) {
                            rpart[l] = make_double2(r0, r1);
                        } else {
                            ss += r0 * r0 + r1 * r1;
                            s1 += r0 + r1;
                        }
                        const size_t o = ro + (size_t)l * NF;
                        nt_store2(a.u + o, un);
                        nt_store2(a.v + o, vn);
                        nt_store2(a.w + o, wn);
                        nt_store2(a.p + o, pc);
                    }
                    prev[l] = pc;
                    pym = pc;
                }
                // keep the next batch's loads after this batch's stores
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        __syncthreads();   // the next step overwrites the tile
    }
    double s2 = 0.0;
    block_sum3<NTHR>(ss, s1, s2, sred);
    if (threadIdx.x == 0) {
        a.partials[3 * blockIdx.x] = ss;
        a.partials[3 * blockIdx.x + 1] = s1;
        a.partials[3 * blockIdx.x + 2] = 0.0;
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

template <typename T, int EMAX, int NTHR, int NF, int PS = kPadShift>
__global__ __launch_bounds__(NTHR) void k_yfwd(YArgs<T> a) {
    __shared__ T sre[lds_elems(EMAX, PS)];
    __shared__ T sim[lds_elems(EMAX, PS)];
    constexpr int NSF = NF > 0 ? tile_nseq(EMAX, NF, PS) : 0;
    const int N = NF > 0 ? NF : a.ny;
    const int SP = seq_stride(N, PS);
    const int nx = a.nx;
    const int nseq = NF > 0 ? NSF : a.nseq;
    const int TX = 2 * nseq;
    // tiles in XCD-contiguous runs (measured: 8-20 % faster at 512 and 768;
    // with 64-byte tile rows the two tiles sharing each 128-byte line also
    // meet in one L2)
    const int bx = (int)xcd_remap(blockIdx.x, gridDim.x);
    const int k = bx / a.ntile;
    const int tile = bx - k * a.ntile;
    const int i0 = tile * TX;
    T* __restrict__ d = a.data + (size_t)k * nx * N + i0;
    // Fixed path: the post-twiddles cos, sin (pi m / 2NF) of the output rows
    // are read before the tile, unconditionally (the tables exist for both
    // boundary kinds; a periodic line ignores them): a table load between
    // the stores would make every store wait for the previous one.  FP64
    // keeps them in registers and its FFT twiddles' round trip overlaps the
    // tile loads; FP32 tiles, whose second workgroup per CU allows no extra
    // registers (1024 threads, at most 64 VGPRs), stage both tables in LDS
    // first (post-twiddles at 2 NF and 3 NF; the launcher sizes the dynamic
    // LDS).
    constexpr bool TL = NF > 0 && sizeof(T) == 4;
    T* twl = lds_twiddle_ptr<T>();
    TwiddleRegs<T, NTHR, ((NF > 0 && !TL) ? NF : 1)> twr;
    if constexpr (NF == 0 || TL) stage_twiddles<T, NTHR>(twl, a.twc, a.tws, N);
    if constexpr (TL) stage_twiddles<T, NTHR>(twl + 2 * NF, a.dctc, a.dcts, NF);
    if constexpr (NF > 0 && !TL) twr.load(a.twc, a.tws);
    constexpr int YP = (NF > 0 && !TL) ? NF / (NTHR / (NSF > 0 ? NSF : 1)) : 1;
    T wr[YP], wi[YP];
    if constexpr (NF > 0) {
        // lane: column pair s (= sequence s), rows jr + r * RPP
        using V2 = typename Vec2T<T>::type;
        constexpr int RPP = NTHR / NSF, NPASS = NF / RPP;
        static_assert(NTHR % NSF == 0 && NF % RPP == 0 && RPP % 2 == 0, "fixed y tile");
        const int s = threadIdx.x % NSF, jr = threadIdx.x / NSF;
        const unsigned lo = (unsigned)(jr * nx + 2 * s);
        if constexpr (!TL) {
#pragma unroll
            for (int r = 0; r < NPASS; ++r) {
                const int m = jr + r * RPP;
                wr[r] = a.dctc[m];
                wi[r] = a.dcts[m];
            }
        }
        V2 val[NPASS];
#pragma unroll
        for (int r = 0; r < NPASS; ++r) val[r] = *reinterpret_cast<const V2*>(d + (size_t)(r * RPP) * nx + lo);
        // keep the post-twiddles in registers from here on (the compiler
        // would otherwise reload each next to its use, one wait per row)
        if constexpr (!TL) {
#pragma unroll
            for (int r = 0; r < NPASS; ++r) asm volatile("" : "+v"(wr[r]), "+v"(wi[r]));
            twr.store(twl);
        }
#pragma unroll
        for (int r = 0; r < NPASS; ++r) {
            const int j = jr + r * RPP;
            const int o = s * SP + li<PS>(0, (a.bcy == FSEI_BC_WALL) ? mk_pos(j, NF) : j, SP);
            sre[o] = val[r].x;
            sim[o] = val[r].y;
        }
    } else {
        constexpr int PLD = 2 * EMAX / NTHR;
        T val[PLD];
#pragma unroll
        for (int r = 0; r < PLD; ++r) {
            const int e = threadIdx.x + r * NTHR;
            const int j = e / TX;
            const int c = e - j * TX;
            val[r] = (e < TX * N && i0 + c < nx) ? d[j * nx + c] : (T)0;
        }
#pragma unroll
        for (int r = 0; r < PLD; ++r) {
            const int e = threadIdx.x + r * NTHR;
            if (e < TX * N) {
                const int j = e / TX;
                const int c = e - j * TX;
                const int n = (a.bcy == FSEI_BC_WALL) ? mk_pos(j, N) : j;
                if (c & 1) sim[li<PS>(c >> 1, n, SP)] = val[r];
                else sre[li<PS>(c >> 1, n, SP)] = val[r];
            }
        }
    }
    __syncthreads();
    fft_lds<T, EMAX, NTHR, -1, NF, PS>(sre, sim, N, nseq, a.fp, twl, twl + N);
    if constexpr (NF > 0) {
        using V2 = typename Vec2T<T>::type;
        constexpr int RPP = NTHR / NSF, NPASS = NF / RPP;
        const int s = threadIdx.x % NSF, mr = threadIdx.x / NSF;
        const unsigned lo = (unsigned)(mr * nx + 2 * s);
#pragma unroll
        for (int r = 0; r < NPASS; ++r) {
            const int m = mr + r * RPP;
            const int mm = (m == 0) ? 0 : NF - m;
            const int om = s * SP + li<PS>(0, m, SP), omm = s * SP + li<PS>(0, mm, SP);
            V2 res;
            const T cr = TL ? twl[2 * NF + m] : wr[TL ? 0 : r];
            const T sr = TL ? twl[3 * NF + m] : wi[TL ? 0 : r];
            post_fwd_v<T>(a.bcy, 2 * m <= NF, sre[om], sim[om], sre[omm], sim[omm], cr, -sr, res.x, res.y);
            *reinterpret_cast<V2*>(d + (size_t)(r * RPP) * nx + lo) = res;
        }
    } else {
        constexpr int PST = EMAX / NTHR;
#pragma unroll
        for (int r = 0; r < PST; ++r) {
            const int e = threadIdx.x + r * NTHR;
            if (e < nseq * N) {
                const int m = e / nseq;
                const int s = e - m * nseq;
                T xa, xb;
                post_fwd<T, PS>(sre, sim, s, SP, N, m, a.bcy, a.dctc, a.dcts, xa, xb);
                if (i0 + 2 * s < nx) d[m * nx + 2 * s] = xa;
                if (i0 + 2 * s + 1 < nx) d[m * nx + 2 * s + 1] = xb;
            }
        }
    }
}

template <typename T, int EMAX, int NTHR, int NF, int PS = kPadShift>
__global__ __launch_bounds__(NTHR) void k_yinv(YArgs<T> a) {
    __shared__ T sre[lds_elems(EMAX, PS)];
    __shared__ T sim[lds_elems(EMAX, PS)];
    constexpr int NSF = NF > 0 ? tile_nseq(EMAX, NF, PS) : 0;
    const int N = NF > 0 ? NF : a.ny;
    const int SP = seq_stride(N, PS);
    const int nx = a.nx;
    const int nseq = NF > 0 ? NSF : a.nseq;
    const int TX = 2 * nseq;
    // tiles in XCD-contiguous runs (measured: 8-20 % faster at 512 and 768;
    // with 64-byte tile rows the two tiles sharing each 128-byte line also
    // meet in one L2)
    const int bx = (int)xcd_remap(blockIdx.x, gridDim.x);
    const int k = bx / a.ntile;
    const int tile = bx - k * a.ntile;
    const int i0 = tile * TX;
    T* __restrict__ d = a.data + (size_t)k * nx * N + i0;
    T* twl = lds_twiddle_ptr<T>();
    TwiddleRegs<T, NTHR, (NF > 0 ? NF : 1)> twr;
    if constexpr (NF == 0) stage_twiddles<T, NTHR>(twl, a.twc, a.tws, N);
    else twr.load(a.twc, a.tws);
    if constexpr (NF > 0) {
        using V2 = typename Vec2T<T>::type;
        constexpr int RPP = NTHR / NSF, NPASS = NF / RPP;
        static_assert(NTHR % NSF == 0 && NF % RPP == 0 && RPP % 2 == 0, "fixed y tile");
        const int s = threadIdx.x % NSF, mr = threadIdx.x / NSF;
        const unsigned lo = (unsigned)(2 * s);
        // each lane loads rows m < NF/2 and its partner NF - m once and
        // forms both pre-twiddled values (m = 0 pairs with NF/2; both
        // of those use only their own row)
        constexpr int NH = NPASS / 2;
        static_assert(NPASS % 2 == 0, "paired rows");
        // pre-twiddles cos/sin(pi m / 2NF) of rows m, loaded before the data
        // and unconditionally (a periodic line ignores them; at NF - m they
        // are sin/cos at m; m = 0 pairs with NF/2)
        T c[NH], sn[NH];
#pragma unroll
        for (int r = 0; r < NH; ++r) {
            const int m = mr + r * RPP;
            c[r] = a.dctc[m];
            sn[r] = a.dcts[m];
        }
        const T c0 = a.dctc[NF / 2], s0 = a.dcts[NF / 2];
        V2 A[NH], B[NH];
#pragma unroll
        for (int r = 0; r < NH; ++r) {
            const int m = mr + r * RPP;
            const int nm = (m == 0) ? NF / 2 : NF - m;
            A[r] = *reinterpret_cast<const V2*>(d + (size_t)m * nx + lo);
            B[r] = *reinterpret_cast<const V2*>(d + (size_t)nm * nx + lo);
        }
        twr.store(twl);
#pragma unroll
        for (int r = 0; r < NH; ++r) {
            const int m = mr + r * RPP;
            const int nm = (m == 0) ? NF / 2 : NF - m;
            const V2 Am = (m == 0) ? B[r] : A[r];
            const T cp = (m == 0) ? c0 : sn[r], sp = (m == 0) ? s0 : c[r];
            T zr, zi;
            pre_inv_cs<T>(NF, m, a.bcy, A[r].x, B[r].x, A[r].y, B[r].y, c[r], sn[r], zr, zi);
            sre[s * SP + li<PS>(0, m, SP)] = zr;
            sim[s * SP + li<PS>(0, m, SP)] = zi;
            pre_inv_cs<T>(NF, nm, a.bcy, B[r].x, Am.x, B[r].y, Am.y, cp, sp, zr, zi);
            sre[s * SP + li<PS>(0, nm, SP)] = zr;
            sim[s * SP + li<PS>(0, nm, SP)] = zi;
        }
    } else {
        constexpr int PLD = EMAX / NTHR;
#pragma unroll
        for (int r = 0; r < PLD; ++r) {
            const int e = threadIdx.x + r * NTHR;
            if (e < nseq * N) {
                const int m = e / nseq;
                const int s = e - m * nseq;
                const int nm = (m == 0) ? 0 : N - m;
                T xam = 0, xanm = 0, xbm = 0, xbnm = 0;
                if (i0 + 2 * s < nx) {
                    xam = d[m * nx + 2 * s];
                    xanm = d[nm * nx + 2 * s];
                }
                if (i0 + 2 * s + 1 < nx) {
                    xbm = d[m * nx + 2 * s + 1];
                    xbnm = d[nm * nx + 2 * s + 1];
                }
                T zr, zi;
                pre_inv<T>(N, m, a.bcy, xam, xanm, xbm, xbnm, a.dctc, a.dcts, zr, zi);
                sre[li<PS>(s, m, SP)] = zr;
                sim[li<PS>(s, m, SP)] = zi;
            }
        }
    }
    __syncthreads();
    fft_lds<T, EMAX, NTHR, 1, NF, PS>(sre, sim, N, nseq, a.fp, twl, twl + N);
    if constexpr (NF > 0) {
        using V2 = typename Vec2T<T>::type;
        constexpr int RPP = NTHR / NSF, NPASS = NF / RPP;
        const int s = threadIdx.x % NSF, jr = threadIdx.x / NSF;
        const unsigned lo = (unsigned)(jr * nx + 2 * s);
#pragma unroll
        for (int r = 0; r < NPASS; ++r) {
            const int j = jr + r * RPP;
            const int o = s * SP + li<PS>(0, (a.bcy == FSEI_BC_WALL) ? mk_pos(j, NF) : j, SP);
            V2 res;
            res.x = sre[o];
            res.y = sim[o];
            *reinterpret_cast<V2*>(d + (size_t)(r * RPP) * nx + lo) = res;
        }
    } else {
        constexpr int PST = 2 * EMAX / NTHR;
#pragma unroll
        for (int r = 0; r < PST; ++r) {
            const int e = threadIdx.x + r * NTHR;
            if (e < TX * N) {
                const int j = e / TX;
                const int c = e - j * TX;
                if (i0 + c < nx) {
                    const int n = (a.bcy == FSEI_BC_WALL) ? mk_pos(j, N) : j;
                    d[j * nx + c] = (c & 1) ? sim[li<PS>(c >> 1, n, SP)] : sre[li<PS>(c >> 1, n, SP)];
                }
            }
        }
    }
}

}  // namespace dev
}  // namespace fsei
