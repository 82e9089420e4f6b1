// HIP side of the C ABI: workspace upload, kernel launches on the plan's
// stream, precision modes, refinement loop, per-kernel event timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <atomic>
#include <mutex>
#include <type_traits>
#include <vector>

#include "fsei_kernels.h"
#include "fsei_plan.h"
#include "fsei_viscous.h"
#include "fsei_momentum.h"
#include "fsei_ibm.h"

using namespace fsei;
using namespace fsei::dev;

namespace {



const char* kSlotNames[FSEI_NUM_KERNEL_SLOTS] = {
    "xfwd", "yfwd", "zsolve", "yinv", "xinv", "grad", "resid_xfwd", "xinv_acc", "norm", "zero_mode",
    "zsolve_fp64_lines", "resid_norm", "resid", "xfwd_r", "grad_resid", "visc_x", "visc_y", "visc_z", "momentum_rhs", "ib_transfer",
    "xinv_grad", "xinv_grad_resid"};
constexpr int K_ZLIST = 10;
constexpr int K_RESNORM = 11;
constexpr int K_RESID_PAIRS = 12;
constexpr int K_XFWD_R = 13;
constexpr int K_GRAD_RESID = 14;
constexpr int K_VISC_X = 15;
constexpr int K_VISC_Y = 16;
constexpr int K_VISC_Z = 17;
constexpr int K_MOM_RHS = 18;
constexpr int K_IB = 19;
constexpr int K_XINV_GRAD = 20;
constexpr int K_XINV_GRAD_RESID = 21;

struct PendingEv {
    hipEvent_t a, b;
    int slot;
};

struct TimingState {
    std::vector<PendingEv> pending;
    std::vector<hipEvent_t> free_ev;
};

TimingState& tstate(fsei_plan* p) {
    // one state per plan, owned through ev_pool[0]
    if (p->ev_pool.empty()) p->ev_pool.push_back(new TimingState());
    return *static_cast<TimingState*>(p->ev_pool[0]);
}

hipEvent_t get_event(TimingState& ts) {
    if (!ts.free_ev.empty()) {
        hipEvent_t e = ts.free_ev.back();
        ts.free_ev.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

void harvest(fsei_plan* p) {
    TimingState& ts = tstate(p);
    for (auto& pe : ts.pending) {
        (void)hipEventSynchronize(pe.b);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, pe.a, pe.b);
        p->t_ms[pe.slot] += ms;
        p->t_count[pe.slot] += 1;
        ts.free_ev.push_back(pe.a);
        ts.free_ev.push_back(pe.b);
    }
    ts.pending.clear();
}

// Brackets one launch with events when timing is on (on the stream the
// launch goes to: the plan's, or its side stream).
struct Timed {
    fsei_plan* p;
    int slot;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    Timed(fsei_plan* pl, int s, void* stream = nullptr)
        : p(pl), slot(s), st((hipStream_t)(stream ? stream : pl->stream)) {
        if (p->timing) {
            TimingState& ts = tstate(p);
            if (ts.pending.size() > 4096) harvest(p);
            a = get_event(ts);
            b = get_event(ts);
            (void)hipEventRecord(a, st);
        }
    }
    ~Timed() {
        if (p->timing) {
            (void)hipEventRecord(b, st);
            tstate(p).pending.push_back({a, b, slot});
        }
    }
};

template <typename T>
const T* tab(const fsei_plan* p, int id);
template <>
const double* tab<double>(const fsei_plan* p, int id) {
    return reinterpret_cast<const double*>((const char*)p->ws + p->ws_tab_d) + p->tab_off[id];
}
template <>
const float* tab<float>(const fsei_plan* p, int id) {
    return reinterpret_cast<const float*>((const char*)p->ws + p->ws_tab_f) + p->tab_off[id];
}

double* scalars(const fsei_plan* p) { return reinterpret_cast<double*>((char*)p->ws + p->ws_scalars); }
double* partials(const fsei_plan* p) { return reinterpret_cast<double*>((char*)p->ws + p->ws_partials); }
void* field1(const fsei_plan* p) { return (char*)p->ws + p->ws_field; }
void* field2(const fsei_plan* p) { return (char*)p->ws + p->ws_field2; }
void* field3(const fsei_plan* p) { return (char*)p->ws + p->ws_field3; }
void* field4(const fsei_plan* p) { return (char*)p->ws + p->ws_field4; }
int* zlist(const fsei_plan* p) { return reinterpret_cast<int*>((char*)p->ws + p->ws_list); }

int nseq_x(const fsei_plan* p) { return x_nseq(p->nx); }

long xblocks(const fsei_plan* p) {
    const long nl = 2L * nseq_x(p);
    return ((long)p->ny * p->nz + nl - 1) / nl;
}

// pair kernels (gradient, residual norm): lanes own two adjacent x-cells,
// workgroups kPairRows rows of one plane
constexpr int kPairRows = 8;
bool pair_tiles(const fsei_plan* p) { return p->nx % 2 == 0 && p->ny % kPairRows == 0; }
bool aligned16(const void* q) { return reinterpret_cast<uintptr_t>(q) % 16 == 0; }
bool al16(const void* q) { return q == nullptr || aligned16(q); }   // optional pointer

// the fixed-length x kernels (NF = 512 or 768, four sequences = eight rows
// per tile) need every tile of rows full and inside one z-plane
bool x_fixed(const fsei_plan* p) {
    return (p->nx == 512 || p->nx == 768) && nseq_x(p) == 4 && p->ny % (2 * nseq_x(p)) == 0;
}

hipStream_t S(const fsei_plan* p) { return (hipStream_t)p->stream; }

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename TI, typename TO, int PRO>
void launch_xfwd(fsei_plan* p, XFwdArgs<TI, TO> a, int slot) {
    a.nx = p->nx;
    a.ny = p->ny;
    a.nz = p->nz;
    a.bcx = p->bcx;
    a.bcy = p->bcy;
    a.nseq = nseq_x(p);
    a.fp = p->fx;
    a.twc = tab<TO>(p, T_TWX_C);
    a.tws = tab<TO>(p, T_TWX_S);
    a.dctc = tab<TO>(p, T_DCTX_C);
    a.dcts = tab<TO>(p, T_DCTX_S);
    const size_t dyn = 2 * p->nx * sizeof(TO);
    // the fixed path reads and writes every field as aligned column pairs
    const bool al = al16(a.u) && al16(a.v) && al16(a.w) && al16(a.gp) && al16(a.f) && al16(a.p) &&
                    al16(a.p32) && al16(a.out) && al16(a.out_f);
    Timed t(p, slot);
    const dim3 grid((unsigned)xblocks(p));
    if (x_fixed(p) && al && p->nx == 512)
        hipLaunchKernelGGL((k_xfwd<TI, TO, PRO, 2048, 256, 512>), grid, dim3(256), dyn, S(p), a);
    else if (x_fixed(p) && al && p->nx == 768)
        hipLaunchKernelGGL((k_xfwd<TI, TO, PRO, 3072, 384, 768>), grid, dim3(384), dyn, S(p), a);
    else if (x_emax(p->nx) == 3072)
        hipLaunchKernelGGL((k_xfwd<TI, TO, PRO, 3072, 384, 0>), grid, dim3(384), dyn, S(p), a);
    else
        hipLaunchKernelGGL((k_xfwd<TI, TO, PRO, 2048, 256, 0>), grid, dim3(256), dyn, S(p), a);
}

template <typename T, typename TP, int EPI>
void launch_xinv(fsei_plan* p, const T* in, TP* out, int slot, const float* add32 = nullptr, T* keep = nullptr,
                 const double* vsum = nullptr) {
    XInvArgs<T, TP> a{};
    a.add32 = add32;
    a.keep = keep;
    a.vsum = vsum;
    a.vscale = 1.0 / ((double)p->nx * (double)p->ny * p->lz);
    a.nx = p->nx;
    a.ny = p->ny;
    a.nz = p->nz;
    a.bcx = p->bcx;
    a.nseq = nseq_x(p);
    a.fp = p->fx;
    a.in = in;
    a.out = out;
    a.twc = tab<T>(p, T_TWX_C);
    a.tws = tab<T>(p, T_TWX_S);
    a.dctc = tab<T>(p, T_DCTX_C);
    a.dcts = tab<T>(p, T_DCTX_S);
    const size_t dyn = 2 * p->nx * sizeof(T);
    const bool al = al16(in) && al16(out) && al16(add32) && al16(keep);
    Timed t(p, slot);
    const dim3 grid((unsigned)xblocks(p));
    if (x_fixed(p) && al && p->nx == 512)
        hipLaunchKernelGGL((k_xinv<T, TP, EPI, 2048, 256, 512>), grid, dim3(256), dyn, S(p), a);
    else if (x_fixed(p) && al && p->nx == 768)
        hipLaunchKernelGGL((k_xinv<T, TP, EPI, 3072, 384, 768>), grid, dim3(384), dyn, S(p), a);
    else if (x_emax(p->nx) == 3072)
        hipLaunchKernelGGL((k_xinv<T, TP, EPI, 3072, 384, 0>), grid, dim3(384), dyn, S(p), a);
    else
        hipLaunchKernelGGL((k_xinv<T, TP, EPI, 2048, 256, 0>), grid, dim3(256), dyn, S(p), a);
}

// fused x inverse + gradient (FP64): nx of a compiled length, whole 8-row
// tiles, every field 16-byte aligned
bool xg_ok(const fsei_plan* p, const void* in, const void* pout, const void* u, const void* v, const void* w) {
    return (p->nx == 512 || p->nx == 768) && p->ny % kXgRows == 0 && aligned16(in) && al16(pout) &&
           aligned16(u) && aligned16(v) && aligned16(w);
}

// planes per workgroup of the fused x inverse + gradient (the chunk's first
// step re-inverts the plane below it: 1/32 more transform work)
constexpr int kXgPlanes = 32;

void launch_xinv_grad(fsei_plan* p, const double* in, double* pout, double* u, double* v, double* w,
                      bool adjoint, double dt) {
    XInvGradArgs a{};
    a.ny = p->ny;
    a.nz = p->nz;
    a.bcx = p->bcx;
    a.bcy = p->bcy;
    a.kc = kXgPlanes;
    a.in = in;
    a.p = pout;
    a.u = u;
    a.v = v;
    a.w = w;
    if (!adjoint) {
        a.cx = -dt / p->dx;
        a.cy = -dt / p->dy;
        a.sw = -dt;
        a.bk = tab<double>(p, T_INV_H);
        a.gk = tab<double>(p, T_INV_H);
    } else {
        a.cx = 1.0 / p->dx;
        a.cy = 1.0 / p->dy;
        a.sw = 1.0;
        a.bk = tab<double>(p, T_INV_DZ);
        a.gk = tab<double>(p, T_GAM_ADJ);
    }
    a.twc = tab<double>(p, T_TWX_C);
    a.tws = tab<double>(p, T_TWX_S);
    a.dctc = tab<double>(p, T_DCTX_C);
    a.dcts = tab<double>(p, T_DCTX_S);
    const int nchunk = (p->nz + a.kc - 1) / a.kc;
    const dim3 grid((unsigned)((p->ny / kXgRows) * nchunk));
    Timed t(p, K_XINV_GRAD);
    if (p->nx == 768)
        hipLaunchKernelGGL((k_xinv_grad<768>), grid, dim3(xg_threads<768>()), 2 * 768 * sizeof(double), S(p), a);
    else
        hipLaunchKernelGGL((k_xinv_grad<512>), grid, dim3(xg_threads<512>()), 2 * 512 * sizeof(double), S(p), a);
}

// dynamic LDS of the compile-time-length y forward kernel: the FFT twiddles,
// and for FP32 also the DCT post-twiddles
template <typename T>
size_t yfwd_dyn(int nf) { return (sizeof(T) == 4 ? 4 : 2) * (size_t)nf * sizeof(T); }

// first refinement correction fused with the gradient and the convergence
// check (FP32 correction, FP64 p): nx of a compiled length, whole 8-row
// tiles, every field 16-byte aligned; returns the number of partials written
bool xgr_ok(const fsei_plan* p, const void* in, const void* p32, const void* p64, const void* f, const void* u,
            const void* v, const void* w) {
    return (p->nx == 512 || p->nx == 768) && p->ny % kXgRows == 0 && aligned16(in) && aligned16(p32) &&
           aligned16(p64) && aligned16(f) && aligned16(u) && aligned16(v) && aligned16(w);
}

long launch_xinv_grad_resid(fsei_plan* p, const float* in, const float* p32, const double* vsum, double* p64,
                            double* u, double* v, double* w, const double* f, double dt) {
    XInvGradResArgs a{};
    a.ny = p->ny;
    a.nz = p->nz;
    a.bcx = p->bcx;
    a.bcy = p->bcy;
    a.kc = kXgPlanes;
    a.in = in;
    a.p32 = p32;
    a.vsum = vsum;
    a.vscale = 1.0 / ((double)p->nx * (double)p->ny * p->lz);
    a.p = p64;
    a.u = u;
    a.v = v;
    a.w = w;
    a.cx = -dt / p->dx;
    a.cy = -dt / p->dy;
    a.sw = -dt;
    a.bk = tab<double>(p, T_INV_H);
    a.gk = tab<double>(p, T_INV_H);
    a.f = f;
    a.idx2 = 1.0 / (p->dx * p->dx);
    a.idy2 = 1.0 / (p->dy * p->dy);
    a.za = tab<double>(p, T_ZA);
    a.zc = tab<double>(p, T_ZC);
    a.scal = scalars(p);
    a.partials = partials(p);
    a.twc = tab<float>(p, T_TWX_C);
    a.tws = tab<float>(p, T_TWX_S);
    a.dctc = tab<float>(p, T_DCTX_C);
    a.dcts = tab<float>(p, T_DCTX_S);
    const int nchunk = (p->nz + a.kc - 1) / a.kc;
    const long nb = (long)(p->ny / kXgRows) * nchunk;
    Timed t(p, K_XINV_GRAD_RESID);
    if (p->nx == 768)
        hipLaunchKernelGGL((k_xinv_grad_resid<768>), dim3((unsigned)nb), dim3(xgr_threads<768>()),
                           2 * 768 * sizeof(float), S(p), a);
    else
        hipLaunchKernelGGL((k_xinv_grad_resid<512>), dim3((unsigned)nb), dim3(xgr_threads<512>()),
                           2 * 512 * sizeof(float), S(p), a);
    return nb;
}

template <typename T, int EMAX, int NTHR>
void launch_y_cfg(fsei_plan* p, YArgs<T> a, bool inverse) {
    a.nseq = std::max(1, std::min(tile_nseq(EMAX, p->ny), (p->nx + 1) / 2));
    // whole 128-byte row segments per tile where the tile holds at least one
    // (16 doubles / 32 floats = 8 / 16 column pairs)
    constexpr int kSeqLine = 64 / (int)sizeof(T);
    if (a.nseq > kSeqLine) a.nseq -= a.nseq % kSeqLine;
    const int tx = 2 * a.nseq;
    a.ntile = (p->nx + tx - 1) / tx;
    const unsigned nb = (unsigned)(a.ntile * p->nz);
    const size_t dyn = 2 * p->ny * sizeof(T);
    // fixed-length variant: full tiles of the compile-time width, column
    // pairs addressed as one aligned vector
    constexpr int kPsF = yfwd_pad<T>();
    // (an FP64 512 line always takes the 4096-element tile: the wider FP64
    // configuration is not compiled for it)
    constexpr bool kFix = y_fixed_ok(EMAX, NTHR, 512) && y_fixed_ok(EMAX, NTHR, 512, kPsF) &&
                          tile_nseq(EMAX, 512, kPsF) == tile_nseq(EMAX, 512) &&
                          (sizeof(T) == 4 || EMAX <= 4096);
    const bool fix = kFix && p->ny == 512 && a.nseq == tile_nseq(EMAX, 512) && p->nx % tx == 0 &&
                     reinterpret_cast<uintptr_t>(a.data) % (2 * sizeof(T)) == 0;
    if (inverse) {
        Timed t(p, K_YINV);
        if constexpr (kFix) {
            if (fix) {
                hipLaunchKernelGGL((k_yinv<T, EMAX, NTHR, 512>), dim3(nb), dim3(NTHR), dyn, S(p), a);
                return;
            }
        }
        hipLaunchKernelGGL((k_yinv<T, EMAX, NTHR, 0>), dim3(nb), dim3(NTHR), dyn, S(p), a);
    } else {
        Timed t(p, K_YFWD);
        if constexpr (kFix) {
            if (fix) {
                hipLaunchKernelGGL((k_yfwd<T, EMAX, NTHR, 512, kPsF>), dim3(nb), dim3(NTHR), yfwd_dyn<T>(512), S(p),
                                   a);
                return;
            }
        }
        hipLaunchKernelGGL((k_yfwd<T, EMAX, NTHR, 0>), dim3(nb), dim3(NTHR), dyn, S(p), a);
    }
}

// Compile-time length 768 in y: tiles of 64-byte row segments (4 FP64 /
// 8 FP32 column pairs) in 768-thread workgroups, two workgroups per CU
// (measured at 768 x 768 x 1024: 5-12 % faster than one workgroup of
// 128-byte segments per CU, whose 105 KB tile leaves no second one room);
// needs whole tiles and pair-aligned data.  Returns false where it does not
// apply.
template <typename T>
bool launch_y768(fsei_plan* p, YArgs<T> a, bool inverse) {
    constexpr int NF = 768, NTHR = 768;
    constexpr int EMAX = (32 / (int)sizeof(T)) * NF;   // 64-B tile rows
    constexpr int kPsF = yfwd_pad<T>();
    static_assert(y_fixed_ok(EMAX, NTHR, NF) && y_fixed_ok(EMAX, NTHR, NF, kPsF) &&
                      tile_nseq(EMAX, NF, kPsF) == tile_nseq(EMAX, NF) && tile_nseq(EMAX, NF) == EMAX / NF,
                  "768 y tile");
    constexpr int NSF = EMAX / NF;
    if (p->ny != NF || p->nx % (2 * NSF) != 0 || reinterpret_cast<uintptr_t>(a.data) % (2 * sizeof(T)) != 0)
        return false;
    a.nseq = NSF;
    a.ntile = p->nx / (2 * NSF);
    const unsigned nb = (unsigned)(a.ntile * p->nz);
    const size_t dyn = 2 * NF * sizeof(T);
    if (inverse) {
        Timed t(p, K_YINV);
        hipLaunchKernelGGL((k_yinv<T, EMAX, NTHR, NF>), dim3(nb), dim3(NTHR), dyn, S(p), a);
    } else {
        Timed t(p, K_YFWD);
        hipLaunchKernelGGL((k_yfwd<T, EMAX, NTHR, NF, kPsF>), dim3(nb), dim3(NTHR), yfwd_dyn<T>(NF), S(p), a);
    }
    return true;
}

// y tiles: the workgroup's LDS holds enough columns that every row segment
// it loads or stores covers 128 B (16 doubles / 32 floats) when ny allows
template <typename T>
void launch_y(fsei_plan* p, T* data, bool inverse) {
    YArgs<T> a{};
    a.nx = p->nx;
    a.ny = p->ny;
    a.nz = p->nz;
    a.bcy = p->bcy;
    a.fp = p->fy;
    a.data = data;
    a.twc = tab<T>(p, T_TWY_C);
    a.tws = tab<T>(p, T_TWY_S);
    a.dctc = tab<T>(p, T_DCTY_C);
    a.dcts = tab<T>(p, T_DCTY_S);
    if (launch_y768<T>(p, a, inverse)) return;
    // complex elements of a tile whose row segments are 128 B; the tile
    // (2 arrays, padded) plus the 2 ny twiddles must fit in the 160 KB of LDS
    const long want = (long)(64 / sizeof(T)) * p->ny;
    auto fits = [&](long emax) {
        return 2L * lds_elems((int)emax) * (long)sizeof(T) + 2L * p->ny * (long)sizeof(T) <= 160L * 1024;
    };
    if (want <= 2048)
        launch_y_cfg<T, 2048, 256>(p, a, inverse);
    else if (want <= 4096 || !fits(8192))
        launch_y_cfg<T, 4096, 512>(p, a, inverse);
    else
        launch_y_cfg<T, 8192, 1024>(p, a, inverse);
}

// chunking of the z lines: P chunks of exactly L rows (L one of the compiled
// sizes), the last chunk padded with decoupled rows; P <= pmax
// compute units of the current device (cached per device; 256 if the query fails)
int cus_of_current_device() {
    constexpr int kDevs = 64;
    static std::atomic<int> cus[kDevs];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kDevs) return 256;
    int n = cus[dev].load(std::memory_order_relaxed);
    if (n <= 0) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cus[dev].store(n, std::memory_order_relaxed);
    }
    return n;
}

bool choose_chunks(int nz, int pmax, int* L, int* P) {
    static const int sizes[] = {4, 8, 12, 16, 24, 32};
    for (int l : sizes) {
        const int pc = (nz + l - 1) / l;
        if (pc <= pmax) {
            *L = l;
            *P = pc;
            return true;
        }
    }
    return false;
}

template <typename TS, typename TC, int TXL, int NT>
void z_dispatch(fsei_plan* p, ZArgs<TS, TC> a, dim3 grid, int slot) {
    const size_t dyn = 0;
    Timed t(p, slot);
    switch (a.L) {
        case 4: hipLaunchKernelGGL((k_zsolve<TS, TC, TXL, 4, NT>), grid, dim3(NT), dyn, S(p), a); break;
        case 8: hipLaunchKernelGGL((k_zsolve<TS, TC, TXL, 8, NT>), grid, dim3(NT), dyn, S(p), a); break;
        case 12: hipLaunchKernelGGL((k_zsolve<TS, TC, TXL, 12, NT>), grid, dim3(NT), dyn, S(p), a); break;
        case 16: hipLaunchKernelGGL((k_zsolve<TS, TC, TXL, 16, NT>), grid, dim3(NT), dyn, S(p), a); break;
        case 24: hipLaunchKernelGGL((k_zsolve<TS, TC, TXL, 24, NT>), grid, dim3(NT), dyn, S(p), a); break;
        default: hipLaunchKernelGGL((k_zsolve<TS, TC, TXL, 32, NT>), grid, dim3(NT), dyn, S(p), a); break;
    }
}

template <typename TS, typename TC, int M, int TXLM, int NT>
void zv_dispatch(fsei_plan* p, ZArgs<TS, TC> a, dim3 grid) {
    Timed t(p, K_ZSOLVE);
    switch (a.L) {
        case 4: hipLaunchKernelGGL((k_zsolvev<TS, TC, M, TXLM, 4, NT>), grid, dim3(NT), 0, S(p), a); break;
        case 8: hipLaunchKernelGGL((k_zsolvev<TS, TC, M, TXLM, 8, NT>), grid, dim3(NT), 0, S(p), a); break;
        case 12: hipLaunchKernelGGL((k_zsolvev<TS, TC, M, TXLM, 12, NT>), grid, dim3(NT), 0, S(p), a); break;
        case 16: hipLaunchKernelGGL((k_zsolvev<TS, TC, M, TXLM, 16, NT>), grid, dim3(NT), 0, S(p), a); break;
        case 24: hipLaunchKernelGGL((k_zsolvev<TS, TC, M, TXLM, 24, NT>), grid, dim3(NT), 0, S(p), a); break;
        default: hipLaunchKernelGGL((k_zsolvev<TS, TC, M, TXLM, 32, NT>), grid, dim3(NT), 0, S(p), a); break;
    }
}

template <typename TS, typename TC>
ZArgs<TS, TC> zargs(const fsei_plan* p, TS* data, int transposed) {
    ZArgs<TS, TC> a{};
    a.nx = p->nx;
    a.ny = p->ny;
    a.nz = p->nz;
    a.transposed = transposed;
    a.data = data;
    a.scale = (TC)(1.0 / ((double)p->nx * (double)p->ny));
    a.za = tab<TC>(p, T_ZA);
    a.zc = tab<TC>(p, T_ZC);
    a.zb0 = tab<TC>(p, T_ZB0);
    a.dz = tab<TC>(p, T_DZ);
    a.inv_dz = tab<TC>(p, T_INV_DZ);
    a.lamx = tab<TC>(p, T_LAMX);
    a.lamy = tab<TC>(p, T_LAMY);
    a.lamx64 = tab<double>(p, T_LAMX);
    a.lamy64 = tab<double>(p, T_LAMY);
    a.sigma_thr = 0.0;
    return a;
}

// z solve of every mode line of `data` (in place), zero mode included
template <typename TS>
void launch_z(fsei_plan* p, TS* data, int transposed, bool record_mean) {
    constexpr bool F32 = std::is_same<TS, float>::value;
    const int nz = p->nz;
    // Tilings (all do the same arithmetic; chosen by measurement at
    // 512 x 512 x 768 and 768 x 768 x 1024): adjacent modes per lane as one
    // vector where nx allows, at most 32 chunks per line; lines longer than
    // 768 rows (chunks of 32 rows) keep one FP64 mode per lane or take 64
    // FP32 chunks of at most 16 rows, which avoids register spills.
    int L = 0, P = 0;
    const bool c32 = choose_chunks(nz, 32, &L, &P);
    // The near-singular lines and the (0,0) line are disjoint from the lines
    // of the tiled kernel: they run on the plan's side stream (when it has
    // one), concurrently with it, joined before the next step.
    hipStream_t side = p->side_stream ? (hipStream_t)p->side_stream : S(p);
    if (p->side_stream) {
        (void)hipEventRecord((hipEvent_t)p->ev_fork, S(p));
        (void)hipStreamWaitEvent(side, (hipEvent_t)p->ev_fork, 0);
    }
    if constexpr (!F32) {
        ZArgs<double, double> a = zargs<double, double>(p, data, transposed);
        a.sigma_thr = p->sigma_thr;   // the host's threshold, compared in FP64
        if (!transposed && c32 && L == 24 && P == 32 && nz == L * P && p->nx % 32 == 0 && aligned16(data)) {
            // whole 32-mode tiles of 768 rows: the persistent kernel with the
            // next tile's first 12 rows of each chunk staged in LDS (0.84 -> 0.66
            // ms at 512x512x768), one workgroup per CU.  With near-singular
            // lines, 32 CUs are left to their kernel on the side stream: with
            // 8 or 16 left it still waited for the whole z solve (0.09 ms in
            // series); with 32 the z solve takes 0.70 ms and the lines run beside it
            a.L = L;
            a.P = P;
            Timed t(p, K_ZSOLVE);
            const long ntiles = (long)(p->nx / 32) * p->ny;
            const int cus = cus_of_current_device();
            const long want = p->nlist > 0 && cus > 64 ? cus - 32 : cus;
            const unsigned g = (unsigned)(ntiles < want ? ntiles : want);
            hipLaunchKernelGGL((k_zsolvev_pf<double, double, 2, 16, 24, 512, 12>), dim3(g), dim3(512), 0, S(p), a);
        } else if (c32 && L <= 24 && p->nx % 2 == 0) {
            a.L = L;
            a.P = P;
            zv_dispatch<double, double, 2, 16, 512>(p, a, dim3((p->nx / 2 + 15) / 16, p->ny));
        } else if (c32) {
            a.L = L;
            a.P = P;
            z_dispatch<double, double, 16, 512>(p, a, dim3((p->nx + 15) / 16, p->ny), K_ZSOLVE);
        } else {
            choose_chunks(nz, 64, &L, &P);
            a.L = L;
            a.P = P;
            z_dispatch<double, double, 8, 512>(p, a, dim3((p->nx + 7) / 8, p->ny), K_ZSOLVE);
        }
    } else {
        ZArgs<float, float> a = zargs<float, float>(p, data, transposed);
        a.sigma_thr = p->sigma_thr;   // the host's threshold, compared in FP64
        if (!transposed && c32 && L == 24 && P == 32 && nz == L * P && p->nx % 64 == 0 && aligned16(data)) {
            // whole 64-mode tiles (256-B rows) of 768 rows: the persistent
            // kernel, one workgroup per CU, the next tile's first 12 rows of each
            // chunk staged in LDS (0.39 -> 0.375 ms at 512x512x768 against the
            // two-workgroup 128-B tiling below); CUs left to the near-singular
            // lines as in FP64
            a.L = L;
            a.P = P;
            Timed t(p, K_ZSOLVE);
            const long ntiles = (long)(p->nx / 64) * p->ny;
            const int cus = cus_of_current_device();
            const long want = p->nlist > 0 && cus > 64 ? cus - 32 : cus;
            const unsigned g = (unsigned)(ntiles < want ? ntiles : want);
            hipLaunchKernelGGL((k_zsolvev_pf<float, float, 4, 16, 24, 512, 12>), dim3(g), dim3(512), 0, S(p), a);
        } else if (c32 && L <= 24 && p->nx % 4 == 0) {
            a.L = L;
            a.P = P;
            // 8 lanes x 4 modes (128-B rows) in 256-thread workgroups: two
            // per CU, one solving while the other loads (11 % faster than 16
            // lanes in 512 threads, one per CU, at 512 x 512 x 768; the FP64
            // kernel the other way round, 18 % slower)
            zv_dispatch<float, float, 4, 8, 256>(p, a, dim3((p->nx / 4 + 7) / 8, p->ny));
        } else if (c32 && L <= 24 && p->nx % 2 == 0) {
            a.L = L;
            a.P = P;
            zv_dispatch<float, float, 2, 32, 1024>(p, a, dim3((p->nx / 2 + 31) / 32, p->ny));
        } else if (p->nx % 2 == 0 && choose_chunks(nz, 64, &L, &P)) {
            a.L = L;
            a.P = P;
            zv_dispatch<float, float, 2, 16, 1024>(p, a, dim3((p->nx / 2 + 15) / 16, p->ny));
        } else if (c32) {
            a.L = L;
            a.P = P;
            z_dispatch<float, float, 32, 1024>(p, a, dim3((p->nx + 31) / 32, p->ny), K_ZSOLVE);
        } else {
            choose_chunks(nz, 64, &L, &P);
            a.L = L;
            a.P = P;
            z_dispatch<float, float, 16, 1024>(p, a, dim3((p->nx + 15) / 16, p->ny), K_ZSOLVE);
        }
    }
    if (p->nlist > 0) {
        ZSeqArgs<TS> b{};
        b.nx = p->nx;
        b.nz = nz;
        b.nlist = p->nlist;
        b.transposed = transposed;
        b.stride = (size_t)p->nx * p->ny;
        b.data = data;
        b.list = zlist(p);
        b.ys = reinterpret_cast<double*>((char*)p->ws + p->ws_seq);
        b.cps = b.ys + (size_t)p->nlist * nz;
        b.za = tab<double>(p, T_ZA);
        b.zc = tab<double>(p, T_ZC);
        b.lamx = tab<double>(p, T_LAMX);
        b.lamy = tab<double>(p, T_LAMY);
        b.dz = tab<double>(p, T_DZ);
        b.scale = 1.0 / ((double)p->nx * (double)p->ny);
        Timed t(p, K_ZLIST, side);
        hipLaunchKernelGGL((k_zline_seq<TS>), dim3((unsigned)((p->nlist + 63) / 64)), dim3(64), 0, side, b);
    }
    ZeroArgs<TS> z{};
    z.nz = nz;
    z.transposed = transposed;
    z.stride = (size_t)p->nx * p->ny;
    z.data = data;
    z.scale = 1.0 / ((double)p->nx * (double)p->ny);
    z.lz = p->lz;
    z.dz = tab<double>(p, T_DZ);
    z.inv_dz = tab<double>(p, T_INV_DZ);
    z.h = tab<double>(p, T_H);
    z.scal = record_mean ? scalars(p) : nullptr;
    {
        Timed t(p, K_PREP, side);
        hipLaunchKernelGGL((k_zero_mode<TS>), dim3(1), dim3(256), 0, side, z);
    }
    if (p->side_stream) {
        (void)hipEventRecord((hipEvent_t)p->ev_join, side);
        (void)hipStreamWaitEvent(S(p), (hipEvent_t)p->ev_join, 0);
    }
}

// k_grad_row2 with the smallest workgroup that gives every cell pair of a
// row a lane (np = nx / 2 <= 512 pairs)
template <typename TIO, typename TP, int GJ>
void launch_grad_row2(fsei_plan* p, const GradArgs<TIO, TP>& a, dim3 grid, int np) {
    if (np > 384)
        hipLaunchKernelGGL((k_grad_row2<TIO, TP, 512, GJ>), grid, dim3(512), 0, S(p), a);
    else if (np > 256)
        hipLaunchKernelGGL((k_grad_row2<TIO, TP, 384, GJ>), grid, dim3(384), 0, S(p), a);
    else if (np > 128)
        hipLaunchKernelGGL((k_grad_row2<TIO, TP, 256, GJ>), grid, dim3(256), 0, S(p), a);
    else if (np > 64)
        hipLaunchKernelGGL((k_grad_row2<TIO, TP, 128, GJ>), grid, dim3(128), 0, S(p), a);
    else
        hipLaunchKernelGGL((k_grad_row2<TIO, TP, 64, GJ>), grid, dim3(64), 0, S(p), a);
}

template <typename TIO, typename TP>
void launch_grad(fsei_plan* p, TIO* u, TIO* v, TIO* w, const TP* pr, bool adjoint, double dt) {
    GradArgs<TIO, TP> a{};
    a.nx = p->nx;
    a.ny = p->ny;
    a.nz = p->nz;
    a.bcx = p->bcx;
    a.bcy = p->bcy;
    a.u = u;
    a.v = v;
    a.w = w;
    a.p = pr;
    if (!adjoint) {
        a.cx = (TIO)(-dt / p->dx);
        a.cy = (TIO)(-dt / p->dy);
        a.sw = (TIO)(-dt);
        a.bk = tab<TIO>(p, T_INV_H);
        a.gk = tab<TIO>(p, T_INV_H);
    } else {
        a.cx = (TIO)(1.0 / p->dx);
        a.cy = (TIO)(1.0 / p->dy);
        a.sw = (TIO)1;
        a.bk = tab<TIO>(p, T_INV_DZ);
        a.gk = tab<TIO>(p, T_GAM_ADJ);
    }
    Timed t(p, K_GRAD);
    const bool al = aligned16(u) && aligned16(v) && aligned16(w) && aligned16(pr);
    const int np = p->nx / 2;
    if (p->nx % 2 == 0 && np <= 512 && p->ny % 8 == 0 && al) {
        // one row per workgroup, one cell pair per lane; rows in 16-row
        // tiles when ny allows (fewer re-read halo rows), else 8
        const dim3 grid((unsigned)((long)p->ny * p->nz));
        if (p->ny % 16 == 0)
            launch_grad_row2<TIO, TP, 16>(p, a, grid, np);
        else
            launch_grad_row2<TIO, TP, 8>(p, a, grid, np);
        return;
    }
    hipLaunchKernelGGL((k_grad<TIO, TP>), dim3((unsigned)((long)p->ny * p->nz)), dim3(256), 0, S(p), a);
}

// FP64 residual norm pass of the refinement (partials of sum r^2, sum r,
// sum dz_k p); returns the number of partials written
template <typename TPP>
long launch_resid_pairs(fsei_plan* p, const double* f, const TPP* pr) {
    ResArgs<TPP> a{};
    a.nx = p->nx;
    a.ny = p->ny;
    a.nz = p->nz;
    a.bcx = p->bcx;
    a.bcy = p->bcy;
    a.f = f;
    a.p = pr;
    a.idx2 = 1.0 / (p->dx * p->dx);
    a.idy2 = 1.0 / (p->dy * p->dy);
    a.za = tab<double>(p, T_ZA);
    a.zc = tab<double>(p, T_ZC);
    a.scal = scalars(p);
    a.dz = tab<double>(p, T_DZ);
    a.partials = partials(p);
    const long nb = (long)(p->ny / kPairRows) * p->nz;
    const dim3 grid((unsigned)nb);
    const int np = p->nx / 2;
    Timed t(p, K_RESNORM);
    if (np == 384)
        hipLaunchKernelGGL((k_resid_pairs<384, kPairRows, TPP>), grid, dim3(384), 0, S(p), a);
    else if (np >= 256)
        hipLaunchKernelGGL((k_resid_pairs<256, kPairRows, TPP>), grid, dim3(256), 0, S(p), a);
    else if (np > 64)
        hipLaunchKernelGGL((k_resid_pairs<128, kPairRows, TPP>), grid, dim3(128), 0, S(p), a);
    else
        hipLaunchKernelGGL((k_resid_pairs<64, kPairRows, TPP>), grid, dim3(64), 0, S(p), a);
    return nb;
}

// Gradient correction of (u, v, w) fused with the residual norm partials of
// the iterate p64 (DELTA: the gradient of the correction c32 instead of p64);
// returns the number of partials written
template <bool DELTA>
long launch_grad_resid(fsei_plan* p, double* u, double* v, double* w, const double* f, const double* p64,
                       const float* c32, double dt) {
    GradResArgs a{};
    a.nx = p->nx;
    a.ny = p->ny;
    a.nz = p->nz;
    a.bcx = p->bcx;
    a.bcy = p->bcy;
    a.u = u;
    a.v = v;
    a.w = w;
    a.p = p64;
    a.c = c32;
    a.cx = -dt / p->dx;
    a.cy = -dt / p->dy;
    a.sw = -dt;
    a.bk = tab<double>(p, T_INV_H);
    a.gk = tab<double>(p, T_INV_H);
    a.f = f;
    a.idx2 = 1.0 / (p->dx * p->dx);
    a.idy2 = 1.0 / (p->dy * p->dy);
    a.za = tab<double>(p, T_ZA);
    a.zc = tab<double>(p, T_ZC);
    a.scal = scalars(p);
    a.partials = partials(p);
    // 16-row tiles halve the re-read halo rows (j-1 of the first row, j+1 of
    // the last) against 8-row tiles when ny allows
    const int rows = (p->ny % 16 == 0) ? 16 : kPairRows;
    const long nb = (long)(p->ny / rows) * p->nz;
    const dim3 grid((unsigned)nb);
    const int np = p->nx / 2;
    Timed t(p, K_GRAD_RESID);
    if (rows == 16) {
        if (np == 384)
            hipLaunchKernelGGL((k_grad_resid<384, 16, DELTA>), grid, dim3(384), 0, S(p), a);
        else if (np >= 256)
            hipLaunchKernelGGL((k_grad_resid<256, 16, DELTA>), grid, dim3(256), 0, S(p), a);
        else if (np > 64)
            hipLaunchKernelGGL((k_grad_resid<128, 16, DELTA>), grid, dim3(128), 0, S(p), a);
        else
            hipLaunchKernelGGL((k_grad_resid<64, 16, DELTA>), grid, dim3(64), 0, S(p), a);
        return nb;
    }
    if (np == 384)
        hipLaunchKernelGGL((k_grad_resid<384, kPairRows, DELTA>), grid, dim3(384), 0, S(p), a);
    else if (np >= 256)
        hipLaunchKernelGGL((k_grad_resid<256, kPairRows, DELTA>), grid, dim3(256), 0, S(p), a);
    else if (np > 64)
        hipLaunchKernelGGL((k_grad_resid<128, kPairRows, DELTA>), grid, dim3(128), 0, S(p), a);
    else
        hipLaunchKernelGGL((k_grad_resid<64, kPairRows, DELTA>), grid, dim3(64), 0, S(p), a);
    return nb;
}

template <typename TI, typename TO>
XFwdArgs<TI, TO> div_args(const fsei_plan* p, const TI* u, const TI* v, const TI* w, const TI* gp, bool adjoint,
                          double dt) {
    XFwdArgs<TI, TO> a{};
    a.u = u;
    a.v = v;
    a.w = w;
    a.gp = gp;
    a.idx = (TI)(1.0 / p->dx);
    a.idy = (TI)(1.0 / p->dy);
    if (!adjoint) {
        a.alpha = (TI)(1.0 / dt);
        a.beta = (TI)0;
        a.zeta = tab<TI>(p, T_INV_DZ);
        a.eta = tab<TI>(p, T_INV_DZ);
    } else {
        a.alpha = (TI)-1;
        a.beta = (TI)(-1.0 / dt);
        a.zeta = tab<TI>(p, T_ZETA_ADJ);
        a.eta = tab<TI>(p, T_INV_H);
    }
    return a;
}

fsei_status check_hip() {
    return (hipGetLastError() == hipSuccess) ? FSEI_OK : FSEI_ERR_HIP;
}

// ---------------------------------------------------------------------------
// implicit viscous step: line solves along x (LDS-staged), y and z (strided)
// ---------------------------------------------------------------------------
template <int L>
void launch_visc_x_L(fsei_plan* p, const ViscArgs& a) {
    const long per = (long)kViscXLines * kViscXTiles;
    const unsigned nb = (unsigned)((a.nlines + per - 1) / per);
    const int dyn = kViscXLines * (a.n + 2) * (int)sizeof(double);
    static bool attr = false;   // allow the tile beyond the default dynamic LDS limit
    if (!attr) {
        (void)hipFuncSetAttribute((const void*)k_visc_x<L>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  kViscXLines * (kViscMaxN + 2) * (int)sizeof(double));
        attr = true;
    }
    hipLaunchKernelGGL((k_visc_x<L>), dim3(nb), dim3(kViscXLines * kViscPmax), dyn, S(p), a);
}

void launch_visc_x(fsei_plan* p, const ViscArgs& a, int L) {
    switch (L) {
        case 4: launch_visc_x_L<4>(p, a); break;
        case 8: launch_visc_x_L<8>(p, a); break;
        case 12: launch_visc_x_L<12>(p, a); break;
        case 16: launch_visc_x_L<16>(p, a); break;
        case 24: launch_visc_x_L<24>(p, a); break;
        default: launch_visc_x_L<32>(p, a); break;
    }
}

template <int M>
void launch_visc_s_M(fsei_plan* p, const ViscArgs& a, int L, unsigned groups) {
    const dim3 g((unsigned)((a.ncol + 16 * M - 1) / (16 * M)), groups);
    const dim3 b(16 * kViscPmax);
    switch (L) {
        case 4: hipLaunchKernelGGL((k_visc_strided<M, 4>), g, b, 0, S(p), a); break;
        case 8: hipLaunchKernelGGL((k_visc_strided<M, 8>), g, b, 0, S(p), a); break;
        case 12: hipLaunchKernelGGL((k_visc_strided<M, 12>), g, b, 0, S(p), a); break;
        case 16: hipLaunchKernelGGL((k_visc_strided<M, 16>), g, b, 0, S(p), a); break;
        case 24: hipLaunchKernelGGL((k_visc_strided<M, 24>), g, b, 0, S(p), a); break;
        default: hipLaunchKernelGGL((k_visc_strided<M, 32>), g, b, 0, S(p), a); break;
    }
}

void launch_visc_strided(fsei_plan* p, const ViscArgs& a, int L, unsigned groups) {
    const bool al = aligned16(a.data) && (a.add == nullptr || aligned16(a.add));
    if (L == 24 && a.n == kViscPmax * 24 && a.ncol % 32 == 0 && al) {
        // whole tiles of 768-row lines: the persistent kernel, the next tile's
        // first 12 rows of each chunk staged in LDS, one workgroup per CU (z
        // pass at 512x512x768: 0.69 -> 0.63 ms per component)
        const int ngx = a.ncol / 32;
        const long ntiles = (long)ngx * groups;
        const int cus = cus_of_current_device();
        const unsigned g = (unsigned)(ntiles < cus ? ntiles : cus);
        hipLaunchKernelGGL((k_visc_strided_pf<24, 12>), dim3(g), dim3(16 * kViscPmax), 0, S(p), a, ngx, (int)ntiles);
        return;
    }
    // two adjacent columns per lane (16-byte accesses) when the rows allow
    if (a.ncol % 2 == 0 && al)
        launch_visc_s_M<2>(p, a, L, groups);
    else
        launch_visc_s_M<1>(p, a, L, groups);
}

fsei_status ready(const fsei_plan* p) {
    if (!p) return FSEI_ERR_ARG;
    if (!p->ws || p->ws_bytes < p->ws_total) return FSEI_ERR_WORKSPACE;
    return FSEI_OK;
}

bool good_dt(double dt) { return std::isfinite(dt) && dt > 0.0; }

fsei_status read_scalars(fsei_plan* p, double* host, int n) {
    if (hipMemcpyAsync(host, scalars(p), n * sizeof(double), hipMemcpyDeviceToHost, S(p)) != hipSuccess)
        return FSEI_ERR_HIP;
    if (hipStreamSynchronize(S(p)) != hipSuccess) return FSEI_ERR_HIP;
    return FSEI_OK;
}

// sums of the last xfwd pass with partials (sum v^2, sum v, sum dz_k v) into
// scalars[off..off+2]; with `vmean`, also scalars[0] = the V-mean of v,
// sum dz_k v / (nx ny lz)
void reduce_partials(fsei_plan* p, int off, bool vmean = false, long nblk = -1) {
    Timed t(p, K_NORM);
    const double scale = 1.0 / ((double)p->nx * (double)p->ny * p->lz);
    if (nblk < 0) nblk = xblocks(p);
    double* out = scalars(p) + off;
    double* mean = vmean ? scalars(p) : nullptr;
    if (nblk <= 4 * kSumGroups) {
        hipLaunchKernelGGL(k_sum_partials<1024>, dim3(1), dim3(1024), 0, S(p), (const double*)partials(p), (int)nblk,
                           out, mean, scale);
        return;
    }
    // two stages: kSumGroups workgroups over contiguous chunks, then one
    // small workgroup over their triples (the group sums follow the
    // partials in the workspace)
    const int chunk = (int)((nblk + kSumGroups - 1) / kSumGroups);
    double* grp = partials(p) + 3 * p->n_partials;
    hipLaunchKernelGGL(k_sum_partials_grp, dim3(kSumGroups), dim3(256), 0, S(p), (const double*)partials(p),
                       (int)nblk, chunk, grp);
    hipLaunchKernelGGL(k_sum_partials<64>, dim3(1), dim3(64), 0, S(p), (const double*)grp, kSumGroups, out, mean,
                       scale);
}

// ---------------------------------------------------------------------------
// FP32 + FP64 iterative refinement.  f (FP64) is the right-hand side; on
// return p64 holds the pressure.
//   p0 = solve32(f); repeat: r = (f - mean) - L p (FP64 stencil), stop when
//   ||r|| <= rtol ||f - mean||, else p += solve32(r).
// ---------------------------------------------------------------------------
// Projection target of a refined solve: with the pair tiling and rtol > 0 the
// gradient correction is fused with the convergence check of each
// correction (the first applies the gradient of p, later ones the gradient of
// their own correction); `applied` tells the caller whether it still has to
// apply the gradient of the final p.
struct RefineGrad {
    double* u;
    double* v;
    double* w;
    double dt;
    bool applied;
};

template <int PRO>
fsei_status refine_solve(fsei_plan* p, XFwdArgs<double, float> first, double* p64, fsei_info* info,
                         RefineGrad* g = nullptr) {
    float* w32 = static_cast<float*>(field2(p));
    double* f64 = static_cast<double*>(field1(p));
    first.out = w32;
    first.out_f = f64;
    first.partials = partials(p);
    first.dzw = tab<double>(p, T_DZ);
    launch_xfwd<double, float, PRO>(p, first, K_XFWD);
    // scalars[5..7] = sum f^2, sum f, sum dz_k f; scalars[0] = V-mean of f in
    // FP64 (the FP32 zero-mode solve removes its own FP32 mean to stay
    // compatible, but the residual must use the exact one: a constant left in
    // the residual is in the null space of L and no correction removes it)
    reduce_partials(p, 5, true);
    launch_y<float>(p, w32, false);
    launch_z<float>(p, w32, 0, false);
    launch_y<float>(p, w32, true);
    // With the pair tiling the first solve's pressure stays in FP32 (its
    // error is FP32-level anyway; the residual is evaluated exactly in FP64
    // from those values and the first correction writes p = p32 + delta in
    // FP64), saving 4 bytes per cell in each of three passes.  Otherwise it is
    // written to p64 directly.
    float* p32 = static_cast<float*>(field4(p));
    const bool pairs = pair_tiles(p) && aligned16(f64) && aligned16(p64) && aligned16(w32) && aligned16(p32);
    if (pairs)
        launch_xinv<float, float, EPI_STORE>(p, w32, p32, K_XINV);
    else
        launch_xinv<float, double, EPI_STORE>(p, w32, p64, K_XINV);
    bool p_in_32 = pairs;   // the current iterate is p32 (before the first correction)
    const double N = (double)p->ncells();
    auto rel_from = [&](const double* h) {
        // ||f - mean||^2 = sum f^2 - 2 mean sum f + N mean^2; h[1] = sum r^2
        const double mean = h[0];
        double fn2 = h[5] - 2.0 * mean * h[6] + N * mean * mean;
        if (fn2 <= 0.0) fn2 = h[5];
        return (fn2 > 0.0) ? std::sqrt(h[1] / fn2) : 0.0;
    };
    XFwdArgs<double, float> r{};
    r.f = f64;
    r.p = p64;
    r.idx2 = 1.0 / (p->dx * p->dx);
    r.idy2 = 1.0 / (p->dy * p->dy);
    r.za = tab<double>(p, T_ZA);
    r.zc = tab<double>(p, T_ZC);
    r.scal = scalars(p);
    r.partials = partials(p);
    r.dzw = tab<double>(p, T_DZ);   // third partial: sum dz_k p of the iterate
    int it = 0;
    double rel = -1.0, rel_prev = -1.0;
    bool converged = false;
    bool floor = false;      // a correction no longer halved the residual
    bool measured = false;   // rel belongs to the current iterate
    long nres = -1;   // partials of the last residual pass (-1: the xfwd tiles)
    // The first solve's residual norm is reduced into scalars[8..10] but not
    // read back on its own: it is fetched with the first corrected iterate's
    // norm, so the common one-correction case waits on the host once.  (A
    // first solve that already meets rtol then still gets one correction.)
    bool first_pending = false;
    double vmean = 0.0;
    auto residual_norm = [&]() -> fsei_status {
        reduce_partials(p, 1, false, nres);   // scalars[1..3]: sum r^2, sum r, (sum dz_k p or 0)
        double h[11];
        fsei_status st = read_scalars(p, h, first_pending ? 11 : 8);
        if (st != FSEI_OK) return st;
        vmean = h[0];
        if (first_pending) {
            double h0[8];
            std::copy(h, h + 8, h0);
            h0[1] = h[8];
            rel = rel_from(h0);
            first_pending = false;
        }
        rel_prev = rel;
        rel = rel_from(h);
        measured = true;
        converged = p->rtol > 0.0 && rel <= p->rtol;
        // the FP64 residual cannot fall below the rounding floor of the
        // stencil applied to this p: stop once a correction gains < 2x
        floor = !converged && rel_prev >= 0.0 && rel > 0.5 * rel_prev;
        return FSEI_OK;
    };
    // Residual passes.  A pass that feeds a correction is the x-forward
    // kernel with the FP64 residual stencil as its prologue (reading the FP32
    // first solve, or the FP64 iterate), writing the FP32 transform of r and
    // the partial sums; a norm-only pass is the pair residual kernel (with
    // the pair tiling) or the same x-forward prologue without output.
    auto norm_pass = [&]() {
        if (pairs) {
            nres = p_in_32 ? launch_resid_pairs(p, f64, (const float*)p32)
                           : launch_resid_pairs(p, f64, (const double*)p64);
        } else {
            r.out = nullptr;
            nres = -1;
            launch_xfwd<double, float, PRO_RESID>(p, r, K_RESNORM);
        }
    };
    auto resid_pass = [&]() {
        nres = -1;
        if (p_in_32) {
            XFwdArgs<double, float> r32 = r;
            r32.p = nullptr;
            r32.p32 = p32;
            r32.out = w32;
            launch_xfwd<double, float, PRO_RESID_F>(p, r32, K_RESID_XFWD);
        } else {
            r.out = w32;
            launch_xfwd<double, float, PRO_RESID>(p, r, K_RESID_XFWD);
        }
    };
    resid_pass();
    if (p->max_iter > 0) {
        // scalars[8..10]: the first solve's sum r^2, sum r and sum dz_k p.
        // The last is its V-integral: the first correction subtracts the
        // V-mean it gives, so p is pinned in FP64 (later corrections are
        // solves of residuals, whose V-mean is zero).
        reduce_partials(p, 8, false, nres);
        first_pending = p->rtol > 0.0;
    } else if (p->rtol > 0.0) {
        fsei_status st = residual_norm();
        if (st != FSEI_OK) return st;
    }
    const double* vsum0 = scalars(p) + 10;
    const bool fuse = g != nullptr && pairs && p->rtol > 0.0 && aligned16(g->u) && aligned16(g->v) &&
                      aligned16(g->w);
    while (!converged && it < p->max_iter) {
        launch_y<float>(p, w32, false);
        launch_z<float>(p, w32, 0, false);
        launch_y<float>(p, w32, true);
        const double* vsum = (it == 0) ? vsum0 : nullptr;
        bool checked = false;   // the gradient and the residual partials of this iterate are done
        if (p_in_32) {
            // p64 = (p32 - its V-mean) + delta; with a projection, in the pass
            // that also applies the gradient of p64 and takes its residual
            if (fuse && xgr_ok(p, w32, p32, p64, f64, g->u, g->v, g->w)) {
                nres = launch_xinv_grad_resid(p, w32, p32, vsum, p64, g->u, g->v, g->w, f64, g->dt);
                g->applied = true;
                checked = true;
            } else {
                launch_xinv<float, double, EPI_ADDF>(p, w32, p64, K_XINV_ACC, p32, nullptr, vsum);
            }
            p_in_32 = false;
        } else if (fuse && g->applied) {
            // p64 += delta, and delta itself kept (in w32) for its gradient
            launch_xinv<float, double, EPI_ACC_KEEP>(p, w32, p64, K_XINV_ACC, nullptr, w32, vsum);
        } else {
            launch_xinv<float, double, EPI_ACC>(p, w32, p64, K_XINV_ACC, nullptr, nullptr, vsum);
        }
        ++it;
        measured = false;
        bool transformed = false;   // the next correction's transformed residual is in w32
        if (p->rtol > 0.0) {
            // convergence check of the corrected iterate: for a projection
            // fused with the gradient correction; for a solve that may take
            // another correction, the residual pass of that correction (its
            // partials are this iterate's norm: r is evaluated once, and the
            // transform is wasted only on the last iteration); else norm only
            if (checked) {
            } else if (fuse) {
                nres = g->applied ? launch_grad_resid<true>(p, g->u, g->v, g->w, f64, p64, w32, g->dt)
                                  : launch_grad_resid<false>(p, g->u, g->v, g->w, f64, p64, nullptr, g->dt);
                g->applied = true;
            } else if (it < p->max_iter) {
                resid_pass();
                transformed = true;
            } else {
                norm_pass();
            }
            fsei_status st = residual_norm();
            if (st != FSEI_OK) return st;
            if (converged || floor) break;
        }
        // residual again, transformed for the next correction
        if (it < p->max_iter && !transformed) resid_pass();
    }
    if (p_in_32) {
        // no correction ran (max_iter = 0, or the first solve already met
        // rtol): the iterate is the FP32 first solve
        const size_t n = p->ncells();
        Timed t(p, K_XINV_ACC);
        hipLaunchKernelGGL(k_widen, dim3((unsigned)std::min<size_t>((n + 255) / 256, 65536)), dim3(256), 0, S(p),
                           (const float*)p32, p64, n);
        p_in_32 = false;
    }
    if (info != nullptr && !measured) {
        norm_pass();
        fsei_status st = residual_norm();
        if (st != FSEI_OK) return st;
    }
    if (info) {
        if (!measured) {
            double h[1];
            fsei_status st = read_scalars(p, h, 1);
            if (st != FSEI_OK) return st;
            vmean = h[0];
        }
        info->iterations = it;
        info->rel_residual = rel;
        info->rhs_vmean_removed = vmean;
        info->floor_reached = floor ? 1 : 0;
    }
    fsei_status st = check_hip();
    if (st != FSEI_OK) return st;
    if (p->rtol > 0.0 && !converged) return FSEI_ERR_NOT_CONVERGED;
    return FSEI_OK;
}

}  // namespace

extern "C" {

void fsei_poisson_plan_destroy(fsei_plan* p) {
    if (!p) return;
    if (!p->ev_pool.empty()) {
        TimingState* ts = static_cast<TimingState*>(p->ev_pool[0]);
        for (auto& pe : ts->pending) {
            (void)hipEventDestroy(pe.a);
            (void)hipEventDestroy(pe.b);
        }
        for (auto e : ts->free_ev) (void)hipEventDestroy(e);
        delete ts;
    }
    if (p->side_stream) {
        (void)hipStreamDestroy((hipStream_t)p->side_stream);
        (void)hipEventDestroy((hipEvent_t)p->ev_fork);
        (void)hipEventDestroy((hipEvent_t)p->ev_join);
    }
    delete p;
}

fsei_status fsei_plan_set_workspace(fsei_plan* p, void* dev, size_t bytes) {
    if (!p || !dev) return FSEI_ERR_ARG;
    if (((uintptr_t)dev % kAlign) != 0 || bytes < p->ws_total) return FSEI_ERR_WORKSPACE;
    if (hipMemcpy((char*)dev + p->ws_tab_d, p->tab_d.data(), p->tab_d.size() * sizeof(double),
                  hipMemcpyHostToDevice) != hipSuccess)
        return FSEI_ERR_HIP;
    if (hipMemcpy((char*)dev + p->ws_tab_f, p->tab_f.data(), p->tab_f.size() * sizeof(float),
                  hipMemcpyHostToDevice) != hipSuccess)
        return FSEI_ERR_HIP;
    if (!p->list_host.empty()) {
        if (hipMemcpy((char*)dev + p->ws_list, p->list_host.data(), p->list_host.size() * sizeof(int),
                      hipMemcpyHostToDevice) != hipSuccess)
            return FSEI_ERR_HIP;
    }
    if (hipMemset((char*)dev + p->ws_scalars, 0, fsei_plan_impl::kScalars * sizeof(double)) != hipSuccess)
        return FSEI_ERR_HIP;
    p->ws = dev;
    p->ws_bytes = bytes;
    for (double& b : p->visc_beta) b = 0.0;   // viscous tables live in the workspace: rebuild on next use
    if (!p->side_stream) {
        // side stream (default priority) and the fork / join events of the z
        // solve; without them everything runs on the plan's stream
        hipStream_t st = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&e0, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&e1, hipEventDisableTiming) == hipSuccess) {
            p->side_stream = st;
            p->ev_fork = e0;
            p->ev_join = e1;
        } else {
            if (st) (void)hipStreamDestroy(st);
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            (void)hipGetLastError();
        }
    }
    return FSEI_OK;
}

fsei_status fsei_plan_set_stream(fsei_plan* p, void* stream) {
    if (!p) return FSEI_ERR_ARG;
    p->stream = stream;
    return FSEI_OK;
}

fsei_status fsei_poisson_solve(fsei_plan* p, const double* f, double* out, fsei_info* info) {
    fsei_status st = ready(p);
    if (st != FSEI_OK) return st;
    if (!f || !out) return FSEI_ERR_ARG;
    if (p->precision == FSEI_PREC_FP32) return FSEI_ERR_PRECISION;
    if (p->precision == FSEI_PREC_FP32_REFINE) {
        XFwdArgs<double, float> a{};
        a.f = f;
        return refine_solve<PRO_COPY>(p, a, out, info);
    }
    XFwdArgs<double, double> a{};
    a.f = f;
    a.out = out;
    launch_xfwd<double, double, PRO_COPY>(p, a, K_XFWD);
    launch_y<double>(p, out, false);
    launch_z<double>(p, out, 0, true);
    launch_y<double>(p, out, true);
    launch_xinv<double, double, EPI_STORE>(p, out, out, K_XINV);
    st = check_hip();
    if (st != FSEI_OK) return st;
    if (info) {
        double h[1];
        st = read_scalars(p, h, 1);
        if (st != FSEI_OK) return st;
        info->iterations = 0;
        info->rel_residual = -1.0;
        info->rhs_vmean_removed = h[0];
        info->floor_reached = 0;
    }
    return FSEI_OK;
}

}  // extern "C"

namespace {

// the projection on the plan's current workspace (arguments checked by the caller)
fsei_status project_impl(fsei_plan* p, double* u, double* v, double* w, double* pout, double dt, fsei_info* info) {
    fsei_status st = FSEI_OK;
    if (p->precision == FSEI_PREC_FP32_REFINE) {
        double* p64 = pout ? pout : static_cast<double*>(field3(p));
        XFwdArgs<double, float> a = div_args<double, float>(p, u, v, w, nullptr, false, dt);
        RefineGrad g{u, v, w, dt, false};
        st = refine_solve<PRO_DIV>(p, a, p64, info, &g);
        if (st != FSEI_OK && st != FSEI_ERR_NOT_CONVERGED) return st;
        if (!g.applied) launch_grad<double, double>(p, u, v, w, p64, false, dt);
        fsei_status st2 = check_hip();
        return (st2 != FSEI_OK) ? st2 : st;
    }
    // the transform chain runs in the workspace field when the x inverse is
    // fused with the gradient (its halo rows must not be overwritten by a
    // neighbouring tile's p), else in the caller's p when given
    double* ws1 = static_cast<double*>(field1(p));
    const bool fused = xg_ok(p, ws1, pout, u, v, w);
    double* buf = (pout && !fused) ? pout : ws1;
    XFwdArgs<double, double> a = div_args<double, double>(p, u, v, w, nullptr, false, dt);
    a.out = buf;
    launch_xfwd<double, double, PRO_DIV>(p, a, K_XFWD);
    launch_y<double>(p, buf, false);
    launch_z<double>(p, buf, 0, true);
    launch_y<double>(p, buf, true);
    if (fused) {
        launch_xinv_grad(p, buf, pout, u, v, w, false, dt);
    } else {
        launch_xinv<double, double, EPI_STORE>(p, buf, buf, K_XINV);
        launch_grad<double, double>(p, u, v, w, buf, false, dt);
    }
    st = check_hip();
    if (st != FSEI_OK) return st;
    if (info) {
        double h[1];
        st = read_scalars(p, h, 1);
        if (st != FSEI_OK) return st;
        info->iterations = 0;
        info->rel_residual = -1.0;
        info->rhs_vmean_removed = h[0];
        info->floor_reached = 0;
    }
    return FSEI_OK;
}

// ---------------------------------------------------------------------------
// Device-resident scratch of the allocation-free projection: one copy per
// GPU, held until the process ends.  Host code never uses the array's name
// as an address: the device address comes from hipGetSymbolAddress, once per
// device, and is kept in scratch_ptr.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)128 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_ptr[kMaxDevices] = {};

__global__ __launch_bounds__(256) void k_zero(double* __restrict__ q, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) q[i] = 0.0;
}

fsei_status scratch_of_current_device(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return FSEI_ERR_HIP;
    if (dev >= kMaxDevices) return FSEI_ERR_HIP;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (scratch_ptr[dev] == nullptr) {
        void* q = nullptr;
        if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || q == nullptr) return FSEI_ERR_HIP;
        scratch_ptr[dev] = q;
    }
    *out = scratch_ptr[dev];
    return FSEI_OK;
}

}  // namespace

extern "C" {

fsei_status fsei_project(fsei_plan* p, double* u, double* v, double* w, double* pout, double dt, fsei_info* info) {
    fsei_status st = ready(p);
    if (st != FSEI_OK) return st;
    if (!u || !v || !w) return FSEI_ERR_ARG;
    if (!good_dt(dt)) return FSEI_ERR_ARG;
    if (p->precision == FSEI_PREC_FP32) return FSEI_ERR_PRECISION;
    return project_impl(p, u, v, w, pout, dt, info);
}

size_t fsei_project_noalloc_max_bytes(void) { return kScratchBytes; }

fsei_status fsei_project_noalloc(fsei_plan* p, double* u, double* v, double* w, double* pout, double dt,
                                 fsei_info* info) {
    if (!p || !u || !v || !w) return FSEI_ERR_ARG;
    if (!good_dt(dt)) return FSEI_ERR_ARG;
    if (p->precision == FSEI_PREC_FP32) return FSEI_ERR_PRECISION;
    if (p->ws_total > kScratchBytes) return FSEI_ERR_SCRATCH;
    void* sp = nullptr;
    fsei_status st = scratch_of_current_device(&sp);
    if (st != FSEI_OK) return st;
    // this plan's tables (and FP64 line list) into the shared scratch, the
    // scalars cleared by a kernel; everything on the plan's stream, so the
    // copies are ordered before the kernels that read them
    hipStream_t s = S(p);
    if (hipMemcpyAsync((char*)sp + p->ws_tab_d, p->tab_d.data(), p->tab_d.size() * sizeof(double),
                       hipMemcpyHostToDevice, s) != hipSuccess)
        return FSEI_ERR_HIP;
    if (hipMemcpyAsync((char*)sp + p->ws_tab_f, p->tab_f.data(), p->tab_f.size() * sizeof(float),
                       hipMemcpyHostToDevice, s) != hipSuccess)
        return FSEI_ERR_HIP;
    if (!p->list_host.empty() &&
        hipMemcpyAsync((char*)sp + p->ws_list, p->list_host.data(), p->list_host.size() * sizeof(int),
                       hipMemcpyHostToDevice, s) != hipSuccess)
        return FSEI_ERR_HIP;
    constexpr int nsc = fsei_plan_impl::kScalars;
    hipLaunchKernelGGL(k_zero, dim3((nsc + 255) / 256), dim3(256), 0, s,
                       reinterpret_cast<double*>((char*)sp + p->ws_scalars), nsc);
    void* ws0 = p->ws;
    const size_t bytes0 = p->ws_bytes;
    p->ws = sp;
    p->ws_bytes = kScratchBytes;
    st = check_hip();
    if (st == FSEI_OK) st = project_impl(p, u, v, w, pout, dt, info);
    p->ws = ws0;
    p->ws_bytes = bytes0;
    return st;
}

fsei_status fsei_project_backward(fsei_plan* p, double* gu, double* gv, double* gw, const double* gp, double dt) {
    fsei_status st = ready(p);
    if (st != FSEI_OK) return st;
    if (!gu || !gv || !gw) return FSEI_ERR_ARG;
    if (!good_dt(dt)) return FSEI_ERR_ARG;
    if (p->precision == FSEI_PREC_FP32) return FSEI_ERR_PRECISION;
    double* buf = static_cast<double*>(field1(p));
    XFwdArgs<double, double> a = div_args<double, double>(p, gu, gv, gw, gp, true, dt);
    a.out = buf;
    launch_xfwd<double, double, PRO_DIV_ADJ>(p, a, K_XFWD);
    launch_y<double>(p, buf, false);
    launch_z<double>(p, buf, 1, false);
    launch_y<double>(p, buf, true);
    if (xg_ok(p, buf, nullptr, gu, gv, gw)) {
        launch_xinv_grad(p, buf, nullptr, gu, gv, gw, true, dt);
    } else {
        launch_xinv<double, double, EPI_STORE>(p, buf, buf, K_XINV);
        launch_grad<double, double>(p, gu, gv, gw, buf, true, dt);
    }
    return check_hip();
}

fsei_status fsei_project_f32(fsei_plan* p, float* u, float* v, float* w, float* pout, float dt) {
    fsei_status st = ready(p);
    if (st != FSEI_OK) return st;
    if (!u || !v || !w) return FSEI_ERR_ARG;
    if (!good_dt(dt)) return FSEI_ERR_ARG;
    if (p->precision != FSEI_PREC_FP32) return FSEI_ERR_PRECISION;
    float* buf = pout ? pout : static_cast<float*>(field1(p));
    XFwdArgs<float, float> a = div_args<float, float>(p, u, v, w, nullptr, false, dt);
    a.out = buf;
    launch_xfwd<float, float, PRO_DIV>(p, a, K_XFWD);
    launch_y<float>(p, buf, false);
    launch_z<float>(p, buf, 0, true);
    launch_y<float>(p, buf, true);
    launch_xinv<float, float, EPI_STORE>(p, buf, buf, K_XINV);
    launch_grad<float, float>(p, u, v, w, buf, false, dt);
    return check_hip();
}

fsei_status fsei_project_backward_f32(fsei_plan* p, float* gu, float* gv, float* gw, const float* gp, float dt) {
    fsei_status st = ready(p);
    if (st != FSEI_OK) return st;
    if (!gu || !gv || !gw) return FSEI_ERR_ARG;
    if (!good_dt(dt)) return FSEI_ERR_ARG;
    if (p->precision != FSEI_PREC_FP32) return FSEI_ERR_PRECISION;
    float* buf = static_cast<float*>(field1(p));
    XFwdArgs<float, float> a = div_args<float, float>(p, gu, gv, gw, gp, true, dt);
    a.out = buf;
    launch_xfwd<float, float, PRO_DIV_ADJ>(p, a, K_XFWD);
    launch_y<float>(p, buf, false);
    launch_z<float>(p, buf, 1, false);
    launch_y<float>(p, buf, true);
    launch_xinv<float, float, EPI_STORE>(p, buf, buf, K_XINV);
    launch_grad<float, float>(p, gu, gv, gw, buf, true, dt);
    return check_hip();
}

static fsei_status viscous_solve(fsei_plan* p, int comp, double* q, double beta, double* add);

fsei_status fsei_viscous_solve(fsei_plan* p, int comp, double* q, double beta) {
    return viscous_solve(p, comp, q, beta, nullptr);
}

fsei_status fsei_viscous_solve_add(fsei_plan* p, int comp, double* rhs, double* u, double beta) {
    if (p && !u) return FSEI_ERR_ARG;
    if (u && u == rhs) return FSEI_ERR_ARG;
    return viscous_solve(p, comp, rhs, beta, u);
}

static fsei_status viscous_solve(fsei_plan* p, int comp, double* q, double beta, double* add) {
    fsei_status st = ready(p);
    if (st != FSEI_OK) return st;
    if (!q || comp < 0 || comp > 2 || !std::isfinite(beta) || !(beta > 0.0)) return FSEI_ERR_ARG;
    if (p->ws_visc_comp == 0) return FSEI_ERR_SIZE;
    double* tab = reinterpret_cast<double*>((char*)p->ws + p->ws_visc + comp * p->ws_visc_comp);
    if (p->visc_beta[comp] != beta) {
        // new tables for this component: drain the stream first so that no
        // earlier solve still reads the old ones, and keep the host copy
        // alive in the plan until the next rebuild (which drains again)
        if (hipStreamSynchronize(S(p)) != hipSuccess) return FSEI_ERR_HIP;
        std::vector<double>& h = p->visc_host[comp];
        h.assign(p->ws_visc_comp / sizeof(double), 0.0);
        build_visc_tables(p, comp, beta, h.data());
        if (hipMemcpyAsync(tab, h.data(), p->ws_visc_comp, hipMemcpyHostToDevice, S(p)) != hipSuccess)
            return FSEI_ERR_HIP;
        p->visc_beta[comp] = beta;
    }
    ViscArgs a{};
    a.data = q;
    // x: contiguous lines
    a.tab = tab;
    a.n = p->nx;
    a.cyc = p->bcx == FSEI_BC_PERIODIC;
    a.nlines = (long)p->ny * p->nz;
    a.vec = (p->nx % 2 == 0 && aligned16(q)) ? 1 : 0;
    {
        Timed t(p, K_VISC_X);
        launch_visc_x(p, a, p->visc_L[0]);
    }
    // y: lines of stride nx inside each z-plane
    a.tab = tab + visc_tab_elems(p->visc_L[0]);
    a.n = p->ny;
    a.cyc = p->bcy == FSEI_BC_PERIODIC;
    a.ncol = p->nx;
    a.rstride = (size_t)p->nx;
    a.bstride = (size_t)p->nx * p->ny;
    a.remap = 1;
    {
        Timed t(p, K_VISC_Y);
        launch_visc_strided(p, a, p->visc_L[1], (unsigned)p->nz);
    }
    // z: lines of stride nx*ny, one group per y row
    a.tab = tab + visc_tab_elems(p->visc_L[0]) + visc_tab_elems(p->visc_L[1]);
    a.n = p->nz;
    a.cyc = 0;
    a.rstride = (size_t)p->nx * p->ny;
    a.bstride = (size_t)p->nx;
    a.remap = 0;
    a.add = add;   // the last pass adds its result to `add` when given
    {
        Timed t(p, K_VISC_Z);
        launch_visc_strided(p, a, p->visc_L[2], (unsigned)p->ny);
    }
    return check_hip();
}

fsei_status fsei_momentum_rhs(fsei_plan* p, const double* u, const double* v, const double* w, double* nu,
                              double* nv, double* nw, double* ru, double* rv, double* rw, double dt, double re,
                              double gamma, double rho) {
    fsei_status st = ready(p);
    if (st != FSEI_OK) return st;
    if (!u || !v || !w || !nu || !nv || !nw || !ru || !rv || !rw) return FSEI_ERR_ARG;
    if (!good_dt(dt) || !std::isfinite(re) || !(re > 0.0) || !std::isfinite(gamma) || !std::isfinite(rho))
        return FSEI_ERR_ARG;
    MomArgs a{};
    a.nx = p->nx;
    a.ny = p->ny;
    a.nz = p->nz;
    a.perx = p->bcx == FSEI_BC_PERIODIC;
    a.pery = p->bcy == FSEI_BC_PERIODIC;
    a.u = u;
    a.v = v;
    a.w = w;
    a.nu = nu;
    a.nv = nv;
    a.nw = nw;
    a.ru = ru;
    a.rv = rv;
    a.rw = rw;
    a.idx = 1.0 / p->dx;
    a.idy = 1.0 / p->dy;
    a.idx2 = a.idx * a.idx;
    a.idy2 = a.idy * a.idy;
    a.dt = dt;
    a.inv_re = 1.0 / re;
    a.gamma = gamma;
    a.rho = rho;
    a.dz = tab<double>(p, T_DZ);
    a.inv_dz = tab<double>(p, T_INV_DZ);
    a.inv_h = tab<double>(p, T_INV_H);
    a.za = tab<double>(p, T_ZA);
    a.zc = tab<double>(p, T_ZC);
    {
        Timed t(p, K_MOM_RHS);
        const unsigned nb = (unsigned)((long)p->ny * p->nz);
        // cell pairs as 16-byte accesses when the rows allow
        const bool pairs = p->nx % 2 == 0 && aligned16(u) && aligned16(v) && aligned16(w) && aligned16(nu) &&
                           aligned16(nv) && aligned16(nw) && aligned16(ru) && aligned16(rv) && aligned16(rw);
        const bool t16 = p->ny % 16 == 0;
        // one wave per row (measured fastest at 512x512x768: 64 lanes 4.49 ms, 128 4.61, 256 5.15),
        // outputs stored non-temporally (nothing re-reads them in this pass)
        if (pairs && t16)
            hipLaunchKernelGGL((k_momentum_rhs_pairs<64, 16, true>), dim3(nb), dim3(64), 0, S(p), a);
        else if (pairs)
            hipLaunchKernelGGL((k_momentum_rhs_pairs<64, 1, true>), dim3(nb), dim3(64), 0, S(p), a);
        else if (t16)
            hipLaunchKernelGGL((k_momentum_rhs<256, 16>), dim3(nb), dim3(256), 0, S(p), a);
        else
            hipLaunchKernelGGL((k_momentum_rhs<256, 1>), dim3(nb), dim3(256), 0, S(p), a);
    }
    return check_hip();
}

fsei_status ib_setup(fsei_plan* p, int comp, const double* xb, long nb, IbArgs* a) {
    fsei_status st = ready(p);
    if (st != FSEI_OK) return st;
    if (comp < 0 || comp > 2 || nb < 0 || (nb > 0 && !xb)) return FSEI_ERR_ARG;
    if (p->nx < 3 || p->ny < 3 || p->nz < 3) return FSEI_ERR_SIZE;
    *a = IbArgs{};
    a->nx = p->nx;
    a->ny = p->ny;
    a->nz = p->nz;
    a->perx = p->bcx == FSEI_BC_PERIODIC;
    a->pery = p->bcy == FSEI_BC_PERIODIC;
    a->comp = comp;
    a->nb = nb;
    a->dx = p->dx;
    a->dy = p->dy;
    a->zn = tab<double>(p, comp == 2 ? T_ZF : T_ZM);
    a->hz = tab<double>(p, comp == 2 ? T_HF : T_DZ);
    a->xb = xb;
    return FSEI_OK;
}

fsei_status fsei_ib_interpolate(fsei_plan* p, int comp, const double* field, const double* xb, long nb,
                                double* ub) {
    IbArgs a;
    fsei_status st = ib_setup(p, comp, xb, nb, &a);
    if (st != FSEI_OK) return st;
    if (nb > 0 && (!field || !ub)) return FSEI_ERR_ARG;
    if (nb == 0) return FSEI_OK;
    a.field = const_cast<double*>(field);
    a.ub = ub;
    {
        Timed t(p, K_IB);
        if (p->ncells() < ((size_t)1 << 32))
            hipLaunchKernelGGL(k_ib_interpolate<uint32_t>, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, S(p), a);
        else
            hipLaunchKernelGGL(k_ib_interpolate<size_t>, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, S(p), a);
    }
    return check_hip();
}

fsei_status fsei_ib_spread(fsei_plan* p, int comp, double* field, const double* xb, const double* fb,
                           const double* dvb, long nb) {
    IbArgs a;
    fsei_status st = ib_setup(p, comp, xb, nb, &a);
    if (st != FSEI_OK) return st;
    if (nb > 0 && (!field || !fb || !dvb)) return FSEI_ERR_ARG;
    if (nb == 0) return FSEI_OK;
    a.field = field;
    a.fb = fb;
    a.dvb = dvb;
    {
        Timed t(p, K_IB);
        if (p->ncells() <= (size_t)0xFFFFFFFEu)   // node offsets fit the LDS table's 32-bit keys
            hipLaunchKernelGGL(k_ib_spread_lds, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, S(p), a);
        else
            hipLaunchKernelGGL(k_ib_spread<size_t>, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, S(p), a);
    }
    return check_hip();
}

fsei_status fsei_plan_set_timing(fsei_plan* p, int enable) {
    if (!p) return FSEI_ERR_ARG;
    p->timing = enable != 0;
    return FSEI_OK;
}

fsei_status fsei_plan_reset_timing(fsei_plan* p) {
    if (!p) return FSEI_ERR_ARG;
    harvest(p);
    for (int s = 0; s < FSEI_NUM_KERNEL_SLOTS; ++s) {
        p->t_ms[s] = 0.0;
        p->t_count[s] = 0;
    }
    return FSEI_OK;
}

fsei_status fsei_plan_kernel_time(fsei_plan* p, int slot, double* total_ms, long* launches, const char** name) {
    if (!p || slot < 0 || slot >= FSEI_NUM_KERNEL_SLOTS) return FSEI_ERR_ARG;
    harvest(p);
    if (total_ms) *total_ms = p->t_ms[slot];
    if (launches) *launches = p->t_count[slot];
    if (name) *name = kSlotNames[slot];
    return FSEI_OK;
}

}  // extern "C"
