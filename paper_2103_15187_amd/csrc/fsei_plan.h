// Internal plan structure shared by the host-only plan code (fsei_plan.cpp)
// and the HIP entry points (fsei_api.hip).  No HIP types appear here, so the
// plan logic builds and runs on a machine without a GPU.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/fsei.h"

namespace fsei {

constexpr int kMaxStages = 16;
constexpr int kMaxN = 2048;     // longest x/y transform
constexpr int kMaxNz = 2048;    // longest z line
constexpr size_t kAlign = 256;
constexpr int kSumGroups = 64;   // first-stage workgroups of the two-stage partial sums
// complex elements per x-transform workgroup (8 per thread; 256 threads, 384
// at length 768 so that the tile holds four sequences there too): small
// tiles keep several workgroups resident per CU so loads, LDS transforms and
// stores of different workgroups overlap
inline int x_emax(int nx) { return nx == 768 ? 3072 : 2048; }

// LDS tile geometry shared by the host (launch sizes) and the kernels:
// sequence s of length N starts at s * seq_stride(N); one array of a tile of
// emax complex elements holds lds_elems(emax) slots.
// One pad slot every 2^ps elements (ps = kPadShift unless a kernel picks its
// own: the best pad depends on the kernel's access pattern and is measured).
constexpr int kPadShift = 4;
constexpr int seq_stride(int N, int ps = kPadShift) { return N + (N >> ps) + 1; }
constexpr int lds_elems(int emax, int ps = kPadShift) { return emax + (emax >> ps) + 16; }
constexpr int tile_nseq(int emax, int N, int ps = kPadShift) {
    return (emax / N < lds_elems(emax, ps) / seq_stride(N, ps)) ? emax / N : lds_elems(emax, ps) / seq_stride(N, ps);
}
inline int x_nseq(int nx) { return tile_nseq(x_emax(nx), nx) > 0 ? tile_nseq(x_emax(nx), nx) : 1; }

// Line solves of the implicit viscous step: every line is cut into
// kViscPmax chunks of L rows (L one of the compiled sizes), so lines of up
// to kViscPmax * 32 rows are supported.  One table block per (component,
// direction) holds visc_tab_elems(L) doubles (layout in fsei_viscous.h).
constexpr int kViscPmax = 32;
constexpr int kViscLv = 5;   // Kogge-Stone levels over the chunks, log2(kViscPmax)
constexpr int kViscMaxN = kViscPmax * 32;
constexpr int visc_tab_elems(int L) { return 6 * kViscPmax * L + 2 * kViscLv * kViscPmax + 2; }
// chunk length for a line of n rows (0: too long)
constexpr int visc_chunk(int n) {
    return n <= kViscPmax * 4    ? 4
           : n <= kViscPmax * 8  ? 8
           : n <= kViscPmax * 12 ? 12
           : n <= kViscPmax * 16 ? 16
           : n <= kViscPmax * 24 ? 24
           : n <= kViscPmax * 32 ? 32
                                 : 0;
}

// Radix schedule of one complex FFT length (radices 8, 4, 2, 3).
struct FftPlan {
    int n = 0;
    int nstages = 0;
    int radix[kMaxStages] = {0};
};

// Names of the per-k / per-mode / twiddle tables stored on the device, each
// in double and in float.  The order is the order inside the table block.
enum TableId {
    T_ZA = 0,      // a_k  = 1/(dz_k h_k), k>=1; a_0 = 0            (nz)
    T_ZC,          // c_k  = 1/(dz_k h_{k+1}), k<=nz-2; c_{nz-1}=0  (nz)
    T_ZB0,         // -(a_k + c_k)                                    (nz)
    T_DZ,          // dz_k                                            (nz)
    T_INV_DZ,      // 1/dz_k                                          (nz)
    T_INV_H,       // 1/h_k, k>=1; 0 at k=0                           (nz)
    T_H,           // h_k = zm_k - zm_{k-1}, k>=1; 0 at k=0          (nz)
    T_ZETA_ADJ,    // 1/h_{k+1} for k<=nz-2, 0 at nz-1                (nz)
    T_GAM_ADJ,     // 1/dz_{k-1} for k>=1, 0 at k=0                   (nz)
    T_ZF,          // z of face k (zc_k), k < nz                     (nz)
    T_ZM,          // z of cell centre k, (zc_k + zc_{k+1})/2         (nz)
    T_HF,          // z extent of the w-face volumes: h_k, k>=1; dz_0/2 (nz)
    T_LAMX,        // modified wavenumbers of x rows                  (nx)
    T_LAMY,        // modified wavenumbers of y rows                  (ny)
    T_TWX_C,       // cos(2 pi t / nx)                                (nx)
    T_TWX_S,       // sin(2 pi t / nx)                                (nx)
    T_DCTX_C,      // cos(pi m / (2 nx))                              (nx)
    T_DCTX_S,      // sin(pi m / (2 nx))                              (nx)
    T_TWY_C,       // cos(2 pi t / ny)                                (ny)
    T_TWY_S,       // sin(2 pi t / ny)                                (ny)
    T_DCTY_C,      // cos(pi m / (2 ny))                              (ny)
    T_DCTY_S,      // sin(pi m / (2 ny))                              (ny)
    T_COUNT
};

// Kernel slots for per-kernel timing.
enum KernelSlot {
    K_XFWD = 0, K_YFWD, K_ZSOLVE, K_YINV, K_XINV, K_GRAD, K_RESID_XFWD, K_XINV_ACC,
    K_NORM, K_PREP, K_SLOT_COUNT
};

struct fsei_plan_impl {
    int nx = 0, ny = 0, nz = 0, bcx = 0, bcy = 0;
    double dx = 0, dy = 0;
    std::vector<double> zc, dz, h;   // h[0] unused (0)
    double lz = 0;
    double dzmin = 0;

    FftPlan fx, fy;

    int precision = FSEI_PREC_FP64;
    double rtol = 1e-10;
    int max_iter = 4;
    double kappa_star = 1e4;

    // host copies of the device tables
    std::vector<double> tab_d;
    std::vector<float> tab_f;
    size_t tab_off[T_COUNT] = {0};   // element offsets inside tab_d / tab_f
    size_t tab_elems = 0;

    // workspace layout (byte offsets)
    size_t ws_tab_d = 0, ws_tab_f = 0, ws_scalars = 0, ws_partials = 0;
    size_t ws_field = 0, ws_field_bytes = 0;       // main intermediate field
    size_t ws_field2 = 0, ws_field2_bytes = 0;     // second field (refine: FP32 work field)
    size_t ws_field3 = 0, ws_field3_bytes = 0;     // refine: FP64 pressure when the caller passes none
    size_t ws_field4 = 0, ws_field4_bytes = 0;     // refine: FP32 pressure of the first solve
    size_t ws_list = 0, ws_list_bytes = 0;         // near-singular mode lines (sequential FP64 solver)
    // implicit viscous step: chunk length per direction (x, y, z; 0 when a
    // line is longer than kViscMaxN), the table blocks of the three
    // components (x, y, z blocks each), and the beta each component's
    // tables were last built for (NaN: not built for this workspace)
    int visc_L[3] = {0, 0, 0};
    size_t ws_visc = 0, ws_visc_comp = 0;           // region offset, bytes per component
    double visc_beta[3] = {0, 0, 0};
    std::vector<double> visc_host[3];
    size_t ws_total = 0;
    size_t n_partials = 0;                          // per-block partial sums (triples)
    static constexpr int kScalars = 64;

    // lines with |lambda_x + lambda_y| < sigma_thr (condition number above
    // kappa_star) are solved one per lane in FP64 with row-sum pivots
    double sigma_thr = 0.0;
    size_t ws_seq = 0;   // FP64 scratch of the near-singular line solver
    std::vector<int> list_host;
    int nlist = 0;

    void* ws = nullptr;
    size_t ws_bytes = 0;
    void* stream = nullptr;
    // side stream of the z solve (near-singular and (0,0) lines run there,
    // concurrently with the tiled lines) and its fork / join events; created
    // with the first workspace, destroyed with the plan
    void* side_stream = nullptr;
    void* ev_fork = nullptr;
    void* ev_join = nullptr;

    // timing
    bool timing = false;
    double t_ms[FSEI_NUM_KERNEL_SLOTS] = {0};
    long t_count[FSEI_NUM_KERNEL_SLOTS] = {0};
    std::vector<void*> ev_pool;          // hipEvent_t pairs, recorded lazily
    std::vector<int> ev_slot;            // pending (start, stop) pairs -> slot
    size_t ev_used = 0;

    size_t ncells() const { return (size_t)nx * ny * nz; }
};

// Host-side helpers (fsei_plan.cpp).
bool factor_radices(int n, FftPlan* out);
void compute_layout(fsei_plan_impl* p);
// Tables of the viscous line solves of component comp (0 u, 1 v, 2 w) for
// beta, x, y and z blocks one after the other (ws_visc_comp bytes).
void build_visc_tables(const fsei_plan_impl* p, int comp, double beta, double* out);

}  // namespace fsei

struct fsei_plan : fsei::fsei_plan_impl {};
