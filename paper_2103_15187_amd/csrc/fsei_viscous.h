// fsei_viscous.h -- batched tridiagonal line solves of the implicit viscous
// step: (I - beta L_d) q = r along one direction d for every line of a field.
//
// Paper, Sec. 2.1 (eq. NSdiscr0: Crank-Nicolson for the viscous term) and
// Sec. 3 (approximate factorisation into one tridiagonal operator per
// direction, Thomas' algorithm, Sherman-Morrison in periodic directions).
//
// Every line of a given component and direction has the same matrix (the
// coefficients depend only on the position along the line), so the whole
// Thomas factorisation is done once on the host and the kernels only run the
// two first-order recurrences of the substitutions,
//
//     d_t = rr_t r_t + al_t d_{t-1}        (forward, al_t = -a_t rr_t)
//     x_t = d_t + cn_t x_{t+1}             (backward, cn_t = -c_t rr_t),
//
// each evaluated in parallel: a line is cut into P chunks of L rows, every
// lane runs its chunk's recurrence from a zero carry, the chunk carries are
// combined by a Kogge-Stone scan over the chunks (the scan multipliers are
// products of al / cn and so are also line-independent tables), and each
// lane adds its carry times the row's product table.  Periodic lines are
// solved on the Sherman-Morrison-modified matrix and corrected by
// x = y - (y_0 + vq y_{n-1}) zt, zt and vq again line-independent.
//
// Tables of one (component, direction), NP = PMAX * L rows (rows >= n are
// padding with every entry 0, so padded rows stay 0 and carry nothing):
//   rr[NP] al[NP] wr[NP] cn[NP] vr[NP] zt[NP] wl[LV*PMAX] vl[LV*PMAX] vq
//   wr_t = prod_{m = chunk start .. t} al_m,  vr_t = prod_{m = t .. chunk end} cn_m,
//   wl / vl = the forward / backward scan multipliers of each level.
#pragma once

#include <hip/hip_runtime.h>

#include "fsei_plan.h"   // kViscPmax, kViscLv, visc_tab_elems
#include "fsei_transforms.h"   // xcd_remap

namespace fsei {
namespace dev {

constexpr int kViscXLines = 8;  // lines per tile of the x kernel
constexpr int kViscXTiles = 4;  // tiles per workgroup of the x kernel

struct ViscArgs {
    double* data;
    const double* tab;
    int n;              // rows of a line
    int cyc;            // periodic line (Sherman-Morrison correction)
    int vec;            // x kernel: n even and data 16-byte aligned (16-byte staging accesses)
    double* add;        // strided kernel: if set, the result is added here (same layout) instead of
                        // stored over data
    int ncol;           // strided kernel: columns (lines side by side along x)
    long nlines;        // x kernel: number of lines
    size_t rstride;     // strided kernel: elements between consecutive rows of a line
    size_t bstride;     // strided kernel: elements between the line groups of blockIdx.y
    int remap;          // strided kernel: workgroups in XCD-contiguous runs (y lines: measured 8 %
                        // faster; z lines: 2 % slower, left in launch order)
};

// Stage the tables of one (component, direction) in LDS.
template <int L, int NT>
__device__ __forceinline__ void visc_load_tables(const double* __restrict__ tab, double* __restrict__ st) {
    constexpr int E = visc_tab_elems(L);
    for (int e = threadIdx.x; e < E; e += NT) st[e] = tab[e];
}

// The same in two steps: every table value of the thread is requested at
// once (load), and written to LDS once the caller has issued its field
// loads (store), so that one round trip covers both.
template <int L, int NT>
struct ViscTabRegs {
    static constexpr int E = visc_tab_elems(L), IT = (E + NT - 1) / NT;
    double v[IT];
    __device__ __forceinline__ void load(const double* __restrict__ tab) {
#pragma unroll
        for (int r = 0; r < IT; ++r) {
            const int e = threadIdx.x + r * NT;
            v[r] = tab[(e < E) ? e : E - 1];
        }
    }
    __device__ __forceinline__ void store(double* __restrict__ st) const {
#pragma unroll
        for (int r = 0; r < IT; ++r) {
            const int e = threadIdx.x + r * NT;
            if (e < E) st[e] = v[r];
        }
    }
};

// Solve the chunks F[h][0..L-1] of M lines held by this lane (chunk p of
// lines owned by lane column `ln`); TXL lanes per chunk row of the
// workgroup, lane index me = p * TXL + ln.  `sc` holds 2 * M * NT scan slots,
// `sx` 2 * M * TXL slots for the periodic correction.  Contains workgroup
// barriers (every lane of the workgroup must call it): fenced ones, or with
// NOFENCE LDS-only ones for callers with direct global-to-LDS loads in
// flight.  `after_fwd()` runs once the forward substitution has used every
// row of F (a no-op for most callers).
struct ViscNoHook {
    __device__ void operator()() const {}
};
template <int M, int L, int TXL, int NT, bool NOFENCE = false, class Hook = ViscNoHook>
__device__ __forceinline__ void visc_core(double (&F)[M][L], int p, int ln, int n, int cyc,
                                          const double* __restrict__ st, double* sc, double* sx,
                                          Hook after_fwd = Hook()) {
    auto sync = [] {
        if constexpr (NOFENCE) sync_lds_nofence();
        else __syncthreads();
    };
    constexpr int NP = kViscPmax * L;
    const double* rr = st;
    const double* al = st + NP;
    const double* wr = st + 2 * NP;
    const double* cn = st + 3 * NP;
    const double* vr = st + 4 * NP;
    const double* zt = st + 5 * NP;
    const double* wl = st + 6 * NP;
    const double* vl = wl + kViscLv * kViscPmax;
    const double vq = vl[kViscLv * kViscPmax];
    const int me = threadIdx.x;
    const int s0 = p * L;
    // forward substitution inside the chunk, zero carry (rows outer: each
    // table value is read once for the M lines)
    double d[M];
#pragma unroll
    for (int h = 0; h < M; ++h) d[h] = 0.0;
#pragma unroll
    for (int t = 0; t < L; ++t) {
        const double r = rr[s0 + t], g = al[s0 + t];
#pragma unroll
        for (int h = 0; h < M; ++h) {
            d[h] = F[h][t] * r + g * d[h];
            F[h][t] = d[h];
        }
    }
    after_fwd();
    // carries of the chunk ends: inclusive scan over the chunks
    double v[M];
#pragma unroll
    for (int h = 0; h < M; ++h) v[h] = F[h][L - 1];
    int ph = 0;
#pragma unroll
    for (int lv = 0; lv < kViscLv; ++lv) {
        const int s = 1 << lv;
        double* b = sc + ph * M * NT;
        ph ^= 1;
#pragma unroll
        for (int h = 0; h < M; ++h) b[M * me + h] = v[h];
        sync();
        if (p >= s) {
            const double m = wl[lv * kViscPmax + p];
#pragma unroll
            for (int h = 0; h < M; ++h) v[h] += m * b[M * (me - s * TXL) + h];
        }
    }
    {
        double* b = sc + ph * M * NT;
        ph ^= 1;
#pragma unroll
        for (int h = 0; h < M; ++h) b[M * me + h] = v[h];
        sync();
        double dprev[M];
#pragma unroll
        for (int h = 0; h < M; ++h) dprev[h] = (p > 0) ? b[M * (me - TXL) + h] : 0.0;
#pragma unroll
        for (int t = 0; t < L; ++t) {
            const double w = wr[s0 + t];
#pragma unroll
            for (int h = 0; h < M; ++h) F[h][t] += w * dprev[h];
        }
    }
    // backward substitution inside the chunk, zero carry
#pragma unroll
    for (int h = 0; h < M; ++h) d[h] = 0.0;
#pragma unroll
    for (int t = L - 1; t >= 0; --t) {
        const double c = cn[s0 + t];
#pragma unroll
        for (int h = 0; h < M; ++h) {
            d[h] = F[h][t] + c * d[h];
            F[h][t] = d[h];
        }
    }
    // carries of the chunk starts: scan from the top
#pragma unroll
    for (int h = 0; h < M; ++h) v[h] = F[h][0];
#pragma unroll
    for (int lv = 0; lv < kViscLv; ++lv) {
        const int s = 1 << lv;
        double* b = sc + ph * M * NT;
        ph ^= 1;
#pragma unroll
        for (int h = 0; h < M; ++h) b[M * me + h] = v[h];
        sync();
        if (p + s < kViscPmax) {
            const double m = vl[lv * kViscPmax + p];
#pragma unroll
            for (int h = 0; h < M; ++h) v[h] += m * b[M * (me + s * TXL) + h];
        }
    }
    {
        double* b = sc + ph * M * NT;
        ph ^= 1;
#pragma unroll
        for (int h = 0; h < M; ++h) b[M * me + h] = v[h];
        sync();
        double xnext[M];
#pragma unroll
        for (int h = 0; h < M; ++h) xnext[h] = (p + 1 < kViscPmax) ? b[M * (me + TXL) + h] : 0.0;
#pragma unroll
        for (int t = 0; t < L; ++t) {
            const double w = vr[s0 + t];
#pragma unroll
            for (int h = 0; h < M; ++h) F[h][t] += w * xnext[h];
        }
    }
    if (cyc) {   // uniform over the workgroup
        const int pl = (n - 1) / L, tl = (n - 1) - pl * L;
        if (p == 0) {
#pragma unroll
            for (int h = 0; h < M; ++h) sx[M * ln + h] = F[h][0];
        }
        if (p == pl) {
            // row tl of the chunk as a masked sum (a selected register index
            // would put F in scratch memory)
#pragma unroll
            for (int h = 0; h < M; ++h) {
                double y = 0.0;
#pragma unroll
                for (int t = 0; t < L; ++t) y += (t == tl) ? F[h][t] : 0.0;
                sx[M * TXL + M * ln + h] = y;
            }
        }
        sync();
        double sm[M];
#pragma unroll
        for (int h = 0; h < M; ++h) sm[h] = sx[M * ln + h] + vq * sx[M * TXL + M * ln + h];
#pragma unroll
        for (int t = 0; t < L; ++t) {
            const double z = zt[s0 + t];
#pragma unroll
            for (int h = 0; h < M; ++h) F[h][t] -= sm[h] * z;
        }
    }
}

// M adjacent values as one native vector
template <int M> struct ViscVec;
template <> struct ViscVec<1> { typedef double type; };
template <> struct ViscVec<2> { typedef double type __attribute__((ext_vector_type(2))); };

// Lines along a strided axis (y: rstride nx, z: rstride nx*ny): TXL lanes x M
// adjacent columns of one line group (blockIdx.y) per workgroup, kViscPmax
// chunks of L rows.  Grid (ceil(ncol / (TXL M)), groups).
template <int M, int L>
__global__ __launch_bounds__(16 * kViscPmax) void k_visc_strided(ViscArgs a) {
    constexpr int TXL = 16, NT = TXL * kViscPmax;
    using V = typename ViscVec<M>::type;
    __shared__ double st[visc_tab_elems(L)];
    __shared__ double sc[2 * M * NT];
    __shared__ double sx[2 * M * TXL];
    ViscTabRegs<L, NT> tr;
    tr.load(a.tab);
    const int ln = threadIdx.x % TXL, p = threadIdx.x / TXL;
    // workgroups in XCD-contiguous runs of (line group, column tile) when asked
    const long vlin = (long)blockIdx.y * gridDim.x + blockIdx.x;
    const long vb = a.remap ? xcd_remap(vlin, (long)gridDim.x * gridDim.y) : vlin;
    const int gy = (int)(vb / gridDim.x), gx = (int)(vb - (long)gy * gridDim.x);
    const int q0 = (gx * TXL + ln) * M;
    const int s0 = p * L;
    const bool full = q0 + M <= a.ncol;
    const bool any = q0 < a.ncol;
    double* __restrict__ base = a.data + (size_t)gy * a.bstride + (any ? q0 : 0);
    double F[M][L];
    // Whole vectors for every lane of the workgroup, else element by element
    // (uniform choice: one load path per row, so the rows' loads are all in
    // flight together)
    const bool wg_full = (gx + 1) * TXL * M <= a.ncol;
    if (wg_full) {
#pragma unroll
        for (int t = 0; t < L; ++t) {
            const int k = s0 + t;
            V v = (V)0.0;
            if (k < a.n) v = *reinterpret_cast<const V*>(base + (size_t)k * a.rstride);
            if constexpr (M == 1) {
                F[0][t] = v;
            } else {
#pragma unroll
                for (int h = 0; h < M; ++h) F[h][t] = v[h];
            }
        }
    } else {
#pragma unroll
        for (int t = 0; t < L; ++t) {
            const int k = s0 + t;
#pragma unroll
            for (int h = 0; h < M; ++h)
                F[h][t] = (k < a.n && q0 + h < a.ncol) ? base[(size_t)k * a.rstride + h] : 0.0;
        }
    }
    tr.store(st);
    __syncthreads();   // tables
    visc_core<M, L, TXL, NT>(F, p, ln, a.n, a.cyc, st, sc, sx);
    if (!any) return;
    // store addresses rebuilt here (not kept live from the loads)
    size_t off = (size_t)gy * a.bstride + q0 + (size_t)s0 * a.rstride;
    asm volatile("" : "+v"(off));
    const bool acc = a.add != nullptr;   // uniform
    base = (acc ? a.add : a.data) + off - (size_t)s0 * a.rstride;
#pragma unroll
    for (int t = 0; t < L; ++t) {
        const int k = s0 + t;
        if (k < a.n) {
            if (full) {
                V v;
                if constexpr (M == 1) {
                    v = F[0][t];
                } else {
#pragma unroll
                    for (int h = 0; h < M; ++h) v[h] = F[h][t];
                }
                V* q = reinterpret_cast<V*>(base + (size_t)k * a.rstride);
                if (acc) v += *q;
                *q = v;
            } else {
#pragma unroll
                for (int h = 0; h < M; ++h)
                    if (q0 + h < a.ncol) {
                        double* q = base + (size_t)k * a.rstride + h;
                        *q = acc ? *q + F[h][t] : F[h][t];
                    }
            }
        }
    }
}

// Persistent form of k_visc_strided for whole tiles: two columns per lane,
// 16 lanes, n = kViscPmax L rows, ncol a multiple of 32, one workgroup per
// CU walking tiles b, b + gridDim.x, ... (tile = (column block, line group)).
// While a tile is solved, the first S rows of every chunk of the next tile
// come into LDS by direct global-to-LDS loads (slot = wave base + lane, so a
// wave reads back only its own slots), issued once the forward substitution
// has used every register row; the solve's barriers are LDS-only.  Same
// arithmetic as k_visc_strided.
template <int L, int S>
__global__ __launch_bounds__(16 * kViscPmax) void k_visc_strided_pf(ViscArgs a, int ngx, int ntiles) {
    constexpr int M = 2, TXL = 16, NT = TXL * kViscPmax;
    using V = typename ViscVec<M>::type;
    static_assert(sizeof(V) == 16 && S >= 1 && S < L, "16-byte rows, prefetched rows");
    typedef __attribute__((address_space(3))) void* lds_void;
    typedef const __attribute__((address_space(1))) void* glb_void;
    __shared__ double st[visc_tab_elems(L)];
    __shared__ double sc[2 * M * NT];
    __shared__ double sx[2 * M * TXL];
    __shared__ V pf[S][NT];
    visc_load_tables<L, NT>(a.tab, st);
    const int ln = threadIdx.x % TXL, p = threadIdx.x / TXL;
    const int s0 = p * L;
    const int wbase = threadIdx.x & ~63;
    // element offset of the lane's first row in tile b
    auto first_row = [&](int b) -> size_t {
        const int gy = b / ngx, gx = b - gy * ngx;
        return (size_t)gy * a.bstride + (size_t)((gx * TXL + ln) * M) + (size_t)s0 * a.rstride;
    };
    auto prefetch = [&](int b) {
        const double* src = a.data + first_row(b);
#pragma unroll
        for (int t = 0; t < S; ++t)
            __builtin_amdgcn_global_load_lds((glb_void)(src + (size_t)t * a.rstride), (lds_void)&pf[t][wbase], 16, 0, 0);
    };
    prefetch(blockIdx.x);   // the host launches at most ntiles workgroups
    __syncthreads();        // tables
    for (int b = blockIdx.x; b < ntiles; b += gridDim.x) {
        // the row stride re-read opaquely each tile: row addresses rebuilt per
        // tile rather than kept live across the loop
        size_t rs = a.rstride;
        asm volatile("" : "+s"(rs));
        const size_t r0 = first_row(b);
        const double* __restrict__ col = a.data + r0;
        double F[M][L];
#pragma unroll
        for (int t = S; t < L; ++t) {
            const V v = *reinterpret_cast<const V*>(col + (size_t)t * rs);
#pragma unroll
            for (int h = 0; h < M; ++h) F[h][t] = v[h];
        }
        // rows 0 .. S-1 from this wave's slots (their direct loads were
        // issued before every load above)
        __builtin_amdgcn_s_waitcnt(imm_wait_vm(L - S));
#pragma unroll
        for (int t = 0; t < S; ++t) {
            const V v = pf[t][threadIdx.x];
#pragma unroll
            for (int h = 0; h < M; ++h) F[h][t] = v[h];
        }
        __builtin_amdgcn_s_waitcnt(imm_wait_lgkm0());   // buffer read: free for the next tile's rows
        const int nb = b + (int)gridDim.x;
        visc_core<M, L, TXL, NT, true>(F, p, ln, a.n, a.cyc, st, sc, sx, [&] {
            __builtin_amdgcn_sched_barrier(0);
            prefetch(nb < ntiles ? nb : b);   // the last tile re-reads its own rows (never used)
            __builtin_amdgcn_sched_barrier(0);
        });
        size_t off = r0;
        asm volatile("" : "+v"(off));
        const bool acc = a.add != nullptr;   // uniform
        double* __restrict__ out = (acc ? a.add : a.data) + off;
#pragma unroll
        for (int t = 0; t < L; ++t) {
            V v;
#pragma unroll
            for (int h = 0; h < M; ++h) v[h] = F[h][t];
            V* q = reinterpret_cast<V*>(out + (size_t)t * rs);
            if (acc) v += *q;
            *q = v;
        }
        sync_lds_nofence();   // sc and sx are rewritten by the next tile
    }
    __builtin_amdgcn_s_waitcnt(0);   // the last direct loads land before the workgroup's LDS is released
}

// Contiguous lines (x): tiles of kViscXLines lines staged through LDS
// (coalesced 16-byte loads and stores when n is even), one lane per (line,
// chunk); each workgroup walks kViscXTiles consecutive tiles so that the
// tables are staged once per kViscXTiles tiles.  Dynamic LDS:
// kViscXLines * (n + 2) doubles.  Grid ceil(nlines / (kViscXLines kViscXTiles)).
template <int L>
__global__ __launch_bounds__(kViscXLines * kViscPmax) void k_visc_x(ViscArgs a) {
    constexpr int TXL = kViscXLines, NT = TXL * kViscPmax;
    constexpr int IPL = (16 * L + NT - 1) / NT;   // 16-byte loads per line and thread (n <= 32 L)
    __shared__ double st[visc_tab_elems(L)];
    __shared__ double sc[2 * NT];
    __shared__ double sx[2 * TXL];
    extern __shared__ __align__(16) unsigned char visc_dyn[];
    double* tile = reinterpret_cast<double*>(visc_dyn);
    visc_load_tables<L, NT>(a.tab, st);
    const int n = a.n, sp = n + 2, h2 = n / 2;
    const bool vec = a.vec != 0;   // uniform
    const int ln = threadIdx.x % TXL, p = threadIdx.x / TXL;
    const int s0 = p * L;
    // 16-byte path: the next tile's loads are issued into registers before
    // the current tile is solved, so they are in flight during the solve
    // (indices clamped into the tile, so every lane loads unconditionally;
    // the clamped values are never stored)
    typedef double d2 __attribute__((ext_vector_type(2)));
    d2 pre[TXL][IPL];
#define FSEI_VISC_FETCH(L0, NL)                                                                        \
    {                                                                                                  \
        const double* __restrict__ gf = a.data + (size_t)(L0) * n;                                     \
        _Pragma("unroll") for (int l = 0; l < TXL; ++l) _Pragma("unroll") for (int r = 0; r < IPL; ++r) { \
            const int lc = (l < (NL)) ? l : (NL) - 1;                                                  \
            int i2 = threadIdx.x + r * NT;                                                             \
            i2 = (i2 < h2) ? i2 : h2 - 1;                                                              \
            pre[l][r] = *reinterpret_cast<const d2*>(gf + (size_t)lc * n + 2 * i2);                    \
        }                                                                                              \
    }
    long line0 = (long)blockIdx.x * kViscXTiles * TXL;
    if (vec && line0 < a.nlines) FSEI_VISC_FETCH(line0, ((a.nlines - line0 < TXL) ? (int)(a.nlines - line0) : TXL))
    // unrolled: the prefetch registers then stay registers across tiles
#pragma unroll
    for (int tt = 0; tt < kViscXTiles; ++tt, line0 += TXL) {
        if (line0 >= a.nlines) break;   // uniform over the workgroup
        const int nl = (a.nlines - line0 < TXL) ? (int)(a.nlines - line0) : TXL;
        double* __restrict__ g = a.data + (size_t)line0 * n;
        __syncthreads();   // the previous tile's stores have read the tile
        if (vec) {
            // every register goes to its (clamped) slot: rows past nl are
            // never read back, a clamped column rewrites its own value
#pragma unroll
            for (int l = 0; l < TXL; ++l)
#pragma unroll
                for (int r = 0; r < IPL; ++r) {
                    int i2 = threadIdx.x + r * NT;
                    i2 = (i2 < h2) ? i2 : h2 - 1;
                    *reinterpret_cast<d2*>(tile + l * sp + 2 * i2) = pre[l][r];
                }
        } else {
            for (int l = 0; l < nl; ++l)
                for (int i = threadIdx.x; i < n; i += NT) tile[l * sp + i] = g[(size_t)l * n + i];
        }
        __syncthreads();   // tile (and, first time, tables) staged
        const long next = line0 + TXL;
        if (vec && tt + 1 < kViscXTiles && next < a.nlines)
            FSEI_VISC_FETCH(next, ((a.nlines - next < TXL) ? (int)(a.nlines - next) : TXL))
        double F[1][L];
#pragma unroll
        for (int t = 0; t < L; ++t) F[0][t] = (s0 + t < n && ln < nl) ? tile[ln * sp + s0 + t] : 0.0;
        visc_core<1, L, TXL, NT>(F, p, ln, n, a.cyc, st, sc, sx);
        if (ln < nl) {
#pragma unroll
            for (int t = 0; t < L; ++t)
                if (s0 + t < n) tile[ln * sp + s0 + t] = F[0][t];
        }
        __syncthreads();
#undef FSEI_VISC_FETCH
        for (int l = 0; l < nl; ++l) {
            if (vec) {
                for (int i = 2 * threadIdx.x; i < n; i += 2 * NT)
                    *reinterpret_cast<double2*>(g + (size_t)l * n + i) =
                        *reinterpret_cast<const double2*>(tile + l * sp + i);
            } else {
                for (int i = threadIdx.x; i < n; i += NT) g[(size_t)l * n + i] = tile[l * sp + i];
            }
        }
    }
}

}  // namespace dev
}  // namespace fsei
