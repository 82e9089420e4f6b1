// fsei_ibm.h -- immersed-boundary moving-least-squares (IB-MLS) transfer
// between Lagrangian markers and one staggered velocity component.
//
// Paper, Sec. 2.1 (eq. interpv, Fig. mls): each marker x_b has a support of
// 3 x 3 x 3 nodes of the component's own lattice; the velocity at the marker
// is sum_k phi_k u_k with moving-least-squares operators on the linear basis
// [1, x, y, z] and an exponential weight centred on the marker; the force
// computed at the marker goes back to the same nodes as a distributed forcing.
//
//     A = sum_k W_k p_k p_k^T,  p_k = [1, x_k - x_b, y_k - y_b, z_k - z_b],
//     phi_k = W_k (A^-1 e_0) . p_k,
//     W_k = exp(-(dx_k/dx)^2 - (dy_k/dy)^2 - (dz_k/hz)^2),
//
// hz the z extent of the support's middle node (cell width for centre
// values, centre distance for w faces).  Supports are the three nodes around
// the nearest one, shifted inwards at walls and wrapped in periodic
// directions (displacements to the nearest periodic image).  One lane per
// marker; A is symmetric positive definite and is factored by Cholesky.
#pragma once

#include <hip/hip_runtime.h>

#include "fsei_plan.h"

namespace fsei {
namespace dev {

struct IbArgs {
    int nx, ny, nz, perx, pery, comp;
    long nb;
    double dx, dy;
    const double* zn;    // z of the component's nodes (faces for w, centres otherwise), nz
    const double* hz;    // z extent of each node's control volume, nz
    const double* xb;    // markers (nb, 3)
    double* field;       // interpolate: read; spread: += (atomic)
    double* ub;          // interpolate: out (nb)
    const double* fb;    // spread: marker values (nb)
    const double* dvb;   // spread: marker volumes (nb)
};

// support along a uniform axis: first index and displacements of its 3 nodes
__device__ __forceinline__ void ib_axis(double xb, double x0, double d, int n, bool per, int (&idx)[3],
                                        double (&dis)[3]) {
    double t = (xb - x0) / d;
    if (!(t == t)) t = 0.0;                       // NaN position: any in-grid support
    t = fmin(fmax(t, -1.0e9), 1.0e9);
    long m = (long)floor(t + 0.5);
    const double L = d * n;
    if (per) {
        m = ((m % n) + n) % n;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int i = (int)((m + q - 1 + n) % n);
            double dd = x0 + i * d - xb;
            dd -= L * rint(dd / L);
            idx[q] = i;
            dis[q] = dd;
        }
    } else {
        m = m < 1 ? 1 : (m > n - 2 ? n - 2 : m);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            idx[q] = (int)(m + q - 1);
            dis[q] = x0 + idx[q] * d - xb;
        }
    }
}

// support along z: nearest node by bisection on the node coordinates
__device__ __forceinline__ int ib_zmid(const double* __restrict__ zn, int n, double zb) {
    int lo = 0, hi = n - 1;   // zn increasing
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (zn[mid] <= zb) lo = mid;
        else hi = mid;
    }
    int m = (fabs(zn[hi] - zb) < fabs(zn[lo] - zb)) ? hi : lo;
    return m < 1 ? 1 : (m > n - 2 ? n - 2 : m);
}

// support of one marker: node indices and marker-node displacements per
// axis, and the z scale of the weight (extent of the middle node's volume)
struct IbSupport {
    int ix[3], iy[3], iz[3];
    double dx[3], dy[3], dz[3];
    double hz;
};

__device__ __forceinline__ IbSupport ib_support(const IbArgs& a, long b) {
    IbSupport s;
    const double xbx = a.xb[3 * b], xby = a.xb[3 * b + 1], xbz = a.xb[3 * b + 2];
    ib_axis(xbx, a.comp == 0 ? 0.0 : 0.5 * a.dx, a.dx, a.nx, a.perx, s.ix, s.dx);
    ib_axis(xby, a.comp == 1 ? 0.0 : 0.5 * a.dy, a.dy, a.ny, a.pery, s.iy, s.dy);
    const int mz = ib_zmid(a.zn, a.nz, (xbz == xbz) ? xbz : 0.0);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        s.iz[q] = mz + q - 1;
        s.dz[q] = a.zn[s.iz[q]] - xbz;
    }
    s.hz = a.hz[mz];
    return s;
}

__device__ __forceinline__ double ib_weight(const IbArgs& a, const IbSupport& s, int ii, int jj, int kk) {
    const double rx = s.dx[ii] / a.dx, ry = s.dy[jj] / a.dy, rz = s.dz[kk] / s.hz;
    return exp(-(rx * rx) - (ry * ry) - (rz * rz));
}

// flat offset of node (ii, jj, kk) of the support; IT: 32-bit offsets when
// the field has fewer than 2^32 cells, else 64-bit
template <typename IT>
__device__ __forceinline__ IT ib_flat(const IbArgs& a, const IbSupport& s, int ii, int jj, int kk) {
    return ((IT)s.iz[kk] * (IT)a.ny + (IT)s.iy[jj]) * (IT)a.nx + (IT)s.ix[ii];
}

// moment matrix A (upper triangle) of the support
struct IbMoments {
    double m00 = 0, m01 = 0, m02 = 0, m03 = 0, m11 = 0, m12 = 0, m13 = 0, m22 = 0, m23 = 0, m33 = 0;
    __device__ __forceinline__ void add(double w, double px, double py, double pz) {
        m00 += w;
        m01 += w * px;
        m02 += w * py;
        m03 += w * pz;
        m11 += w * px * px;
        m12 += w * px * py;
        m13 += w * px * pz;
        m22 += w * py * py;
        m23 += w * py * pz;
        m33 += w * pz * pz;
    }
};

// c = A^-1 e_0 by Cholesky A = L L^T (solve L y = e_0, then L^T c = y); the
// operator of node k is then phi_k = W_k (c0 + c1 dx_k + c2 dy_k + c3 dz_k)
__device__ __forceinline__ void ib_coeffs(const IbMoments& m, double (&c)[4]) {
    const double l00 = sqrt(m.m00);
    const double l10 = m.m01 / l00, l20 = m.m02 / l00, l30 = m.m03 / l00;
    const double l11 = sqrt(m.m11 - l10 * l10);
    const double l21 = (m.m12 - l20 * l10) / l11, l31 = (m.m13 - l30 * l10) / l11;
    const double l22 = sqrt(m.m22 - l20 * l20 - l21 * l21);
    const double l32 = (m.m23 - l30 * l20 - l31 * l21) / l22;
    const double l33 = sqrt(m.m33 - l30 * l30 - l31 * l31 - l32 * l32);
    const double y0 = 1.0 / l00;
    const double y1 = -l10 * y0 / l11;
    const double y2 = -(l20 * y0 + l21 * y1) / l22;
    const double y3 = -(l30 * y0 + l31 * y1 + l32 * y2) / l33;
    c[3] = y3 / l33;
    c[2] = (y2 - l32 * c[3]) / l22;
    c[1] = (y1 - l21 * c[2] - l31 * c[3]) / l11;
    c[0] = (y0 - l10 * c[1] - l20 * c[2] - l30 * c[3]) / l00;
}

// u(x_b) = sum_k phi_k u_k = c0 S0 + c1 S1 + c2 S2 + c3 S3 with
// S = sum_k W_k [1, dx_k, dy_k, dz_k] u_k: the 27 gathers are issued first and
// the weights, moments and value sums formed in one pass while they land
template <typename IT>
__global__ __launch_bounds__(256) void k_ib_interpolate(IbArgs a) {
    const long b = (long)blockIdx.x * 256 + threadIdx.x;
    if (b >= a.nb) return;
    const IbSupport s = ib_support(a, b);
    double val[27];
#pragma unroll
    for (int kk = 0; kk < 3; ++kk)
#pragma unroll
        for (int jj = 0; jj < 3; ++jj)
#pragma unroll
            for (int ii = 0; ii < 3; ++ii) val[(kk * 3 + jj) * 3 + ii] = a.field[ib_flat<IT>(a, s, ii, jj, kk)];
    IbMoments m;
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll
    for (int kk = 0; kk < 3; ++kk)
#pragma unroll
        for (int jj = 0; jj < 3; ++jj)
#pragma unroll
            for (int ii = 0; ii < 3; ++ii) {
                const double w = ib_weight(a, s, ii, jj, kk);
                m.add(w, s.dx[ii], s.dy[jj], s.dz[kk]);
                const double wv = w * val[(kk * 3 + jj) * 3 + ii];
                s0 += wv;
                s1 += wv * s.dx[ii];
                s2 += wv * s.dy[jj];
                s3 += wv * s.dz[kk];
            }
    double c[4];
    ib_coeffs(m, c);
    a.ub[b] = c[0] * s0 + c[1] * s1 + c[2] * s2 + c[3] * s3;
}

// f_k += phi_k F_b dV_b / (dx dy hz_k): moments first, then the weights are
// recomputed (the same arithmetic, so the same values) for the atomic adds,
// so no per-node array stays live
template <typename IT>
__global__ __launch_bounds__(256) void k_ib_spread(IbArgs a) {
    const long b = (long)blockIdx.x * 256 + threadIdx.x;
    if (b >= a.nb) return;
    const IbSupport s = ib_support(a, b);
    IbMoments m;
#pragma unroll
    for (int kk = 0; kk < 3; ++kk)
#pragma unroll
        for (int jj = 0; jj < 3; ++jj)
#pragma unroll
            for (int ii = 0; ii < 3; ++ii) m.add(ib_weight(a, s, ii, jj, kk), s.dx[ii], s.dy[jj], s.dz[kk]);
    double c[4];
    ib_coeffs(m, c);
    const double f = a.fb[b] * a.dvb[b] / (a.dx * a.dy);
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
        const double hk = a.hz[s.iz[kk]];   // control-volume z extent of the plane's nodes
#pragma unroll
        for (int jj = 0; jj < 3; ++jj)
#pragma unroll
            for (int ii = 0; ii < 3; ++ii) {
                const double phi = ib_weight(a, s, ii, jj, kk) * (c[0] + c[1] * s.dx[ii] + c[2] * s.dy[jj] + c[3] * s.dz[kk]);
                atomicAdd(a.field + ib_flat<IT>(a, s, ii, jj, kk), phi * f / hk);
            }
    }
}

// Spreading with the adds of one workgroup's markers combined in LDS first.
// Markers that come in mesh order (neighbours on the surface next to each
// other) share most of their support nodes, so a workgroup's 256 x 27
// contributions land on far fewer distinct nodes.  An open-addressing table
// of kIbSlots (node offset, sum) pairs collects them (bounded linear probing;
// a contribution that finds no slot goes straight to the global atomic), and
// the filled slots are then added to the field, one global atomic each.
// Needs 32-bit offsets: the empty key 0xFFFFFFFF is not a node offset.
constexpr int kIbSlots = 4096;
constexpr int kIbProbes = 8;
constexpr unsigned kIbEmpty = 0xFFFFFFFFu;

__global__ __launch_bounds__(256) void k_ib_spread_lds(IbArgs a) {
    __shared__ unsigned skey[kIbSlots];
    __shared__ double sval[kIbSlots];
    for (int t = threadIdx.x; t < kIbSlots; t += 256) {
        skey[t] = kIbEmpty;
        sval[t] = 0.0;
    }
    __syncthreads();
    const long b = (long)blockIdx.x * 256 + threadIdx.x;
    if (b < a.nb) {
        const IbSupport s = ib_support(a, b);
        IbMoments m;
#pragma unroll
        for (int kk = 0; kk < 3; ++kk)
#pragma unroll
            for (int jj = 0; jj < 3; ++jj)
#pragma unroll
                for (int ii = 0; ii < 3; ++ii) m.add(ib_weight(a, s, ii, jj, kk), s.dx[ii], s.dy[jj], s.dz[kk]);
        double c[4];
        ib_coeffs(m, c);
        const double f = a.fb[b] * a.dvb[b] / (a.dx * a.dy);
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
            const double hk = a.hz[s.iz[kk]];
#pragma unroll
            for (int jj = 0; jj < 3; ++jj)
#pragma unroll
                for (int ii = 0; ii < 3; ++ii) {
                    const double phi =
                        ib_weight(a, s, ii, jj, kk) * (c[0] + c[1] * s.dx[ii] + c[2] * s.dy[jj] + c[3] * s.dz[kk]);
                    const double v = phi * f / hk;
                    const unsigned key = ib_flat<unsigned>(a, s, ii, jj, kk);
                    unsigned h = (key * 2654435761u) >> 20;   // 12 bits: kIbSlots
                    bool done = false;
                    for (int pr = 0; pr < kIbProbes; ++pr) {
                        const unsigned old = atomicCAS(&skey[h], kIbEmpty, key);
                        if (old == kIbEmpty || old == key) {
                            atomicAdd(&sval[h], v);
                            done = true;
                            break;
                        }
                        h = (h + 1) & (kIbSlots - 1);
                    }
                    if (!done) atomicAdd(a.field + key, v);
                }
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kIbSlots; t += 256) {
        const unsigned key = skey[t];
        if (key != kIbEmpty) atomicAdd(a.field + key, sval[t]);
    }
}

}  // namespace dev
}  // namespace fsei
