/*
 * fsei.h -- C ABI of the MI355X pressure-projection library (libfsei.so).
 *
 * The operation (paper, Sec. 2.1, eqs. NS and NSdiscr0): in a fractional-step
 * Navier-Stokes scheme the pressure p^{n+1} is only a Lagrange multiplier that
 * makes the end-of-step velocity divergence free.  Given a provisional
 * velocity u* on a staggered Cartesian mesh (central second-order differences,
 * Sec. 2.1), this library computes
 *
 *     f = D u* / dt,   p = L^+ f   (L = D G),   u = u* - dt G p,
 *
 * with a direct solver: transforms in the two uniform directions x, y (DCT-II
 * for walls, real DFT for periodic), one tridiagonal solve along the
 * stretched wall-normal direction z per (kx, ky) mode, inverse transforms, and
 * the gradient correction.  The zero mode is pinned by the volume-weighted
 * mean, sum_c V_c p_c = 0.
 *
 * Grid and layout (all entry points):
 *   - nx x ny x nz pressure cells; dx, dy uniform; z faces zc[0..nz] strictly
 *     increasing (wall-normal, walls at zc[0] and zc[nz]).
 *   - Every field is a contiguous (nz, ny, nx) array, x fastest, element
 *     (k, j, i) at offset (k*ny + j)*nx + i.
 *   - p[k,j,i] lives at the cell centre; u[k,j,i] on the low x-face of the
 *     cell, v[k,j,i] on the low y-face, w[k,j,i] on the low z-face.
 *   - Wall faces (u[:,:,0] for x walls, v[:,0,:] for y walls, w[0,:,:]
 *     always) are ignored on input and written 0 on output.
 *
 * Memory ownership: all field pointers are HIP device pointers owned by the
 * caller.  The plan owns only host memory.  Device workspace is provided by
 * the caller (fsei_plan_set_workspace) and never freed by the library.
 *
 * Execution: every call enqueues kernels on the plan's stream and returns
 * without waiting, except (a) when an fsei_info pointer is passed (the call
 * then waits for the stream to read back scalars) and (b) FP32_REFINE with
 * rtol > 0 (one scalar is read back per refinement iteration).  Inside the z
 * solve the plan forks to a side stream of its own (created on the current
 * device by fsei_plan_set_workspace, destroyed with the plan) and joins it
 * with events before the next step, so work stays ordered on the plan's
 * stream.  A plan is not thread-safe; calls that share a plan must be
 * serialised by the caller.
 *
 * Errors: arguments are checked before anything is launched; no C++
 * exception crosses this interface.  A failing HIP call is reported as
 * FSEI_ERR_HIP.
 */
#ifndef FSEI_H
#define FSEI_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fsei_plan fsei_plan;

typedef enum {
    FSEI_OK = 0,
    FSEI_ERR_ARG = -1,           /* null pointer, bad enum, non-finite or non-positive scalar */
    FSEI_ERR_SIZE = -2,          /* n < 2, n > 2048, or n not of the form 2^a 3^b (x and y); nz < 2 or nz > 2048 */
    FSEI_ERR_GRID = -3,          /* zc not finite or not strictly increasing; dx or dy <= 0 */
    FSEI_ERR_WORKSPACE = -4,     /* no workspace set, or smaller than fsei_plan_workspace_size, or not 256-B aligned */
    FSEI_ERR_HIP = -5,           /* a HIP runtime call or kernel launch failed */
    FSEI_ERR_NOT_CONVERGED = -6, /* FP32_REFINE did not reach rtol (max_iter corrections done, or the
                                    residual stopped decreasing: fsei_info.floor_reached); outputs hold
                                    the last iterate */
    FSEI_ERR_PRECISION = -7,     /* entry point does not match the plan's precision mode */
    FSEI_ERR_SCRATCH = -8        /* fsei_project_noalloc: the plan's workspace size exceeds the
                                    library's static scratch (fsei_project_noalloc_max_bytes) */
} fsei_status;

/* Boundary condition of the x and y directions (z always has walls). */
enum { FSEI_BC_PERIODIC = 0, FSEI_BC_WALL = 1 };

/* Arithmetic of the solve.
 *   FP64        : every step in double precision.
 *   FP32_REFINE : FP64 input/output; transforms and tridiagonal sweeps in
 *                 FP32 (lines of the near-singular lowest modes in FP64), the
 *                 residual f - L p in FP64, FP32 correction solves until
 *                 ||f - L p||_2 / ||f||_2 <= rtol or max_iter corrections.
 *   FP32        : float input/output, FP32 arithmetic (lowest-mode lines in
 *                 FP64); used by the *_f32 entry points. */
enum { FSEI_PREC_FP64 = 0, FSEI_PREC_FP32_REFINE = 1, FSEI_PREC_FP32 = 2 };

typedef struct {
    int iterations;            /* FP32_REFINE correction solves done (0 otherwise) */
    double rel_residual;       /* ||f - L p||_2 / ||f||_2 when measured (FP32_REFINE), else -1 */
    double rhs_vmean_removed;  /* volume-weighted mean of f removed before the solve */
    int floor_reached;         /* FP32_REFINE: 1 when the refinement stopped because a correction
                                  no longer halved the residual (the FP64 rounding floor of this
                                  right-hand side lies above rtol), else 0 */
} fsei_info;

/* Create a plan (host only; no device memory, no HIP call).
 *   nx, ny : cells in x, y (2 <= n <= 2048, n = 2^a 3^b)
 *   nz     : cells in z (2 <= nz <= 2048)
 *   bc     : bc[0] for x, bc[1] for y, each FSEI_BC_PERIODIC or FSEI_BC_WALL
 *   dx, dy : uniform spacings (> 0)
 *   zc     : HOST array of nz+1 z-face coordinates, strictly increasing; copied
 *   out    : receives the plan (set to NULL on error)
 * Defaults: FP64 precision, null stream, no workspace. */
fsei_status fsei_poisson_plan_create(int nx, int ny, int nz, const int bc[2], double dx, double dy,
                                     const double* zc, fsei_plan** out);

/* Destroy a plan (host memory only; NULL is accepted). */
void fsei_poisson_plan_destroy(fsei_plan* plan);

/* Select the precision mode (FSEI_PREC_*).  rtol >= 0 (0 = run exactly
 * max_iter corrections without reading back residuals); 0 <= max_iter <= 64;
 * both only matter for FP32_REFINE.  Changes the workspace size and layout: a
 * workspace set before is dropped, so call this before
 * fsei_plan_workspace_size / fsei_plan_set_workspace. */
fsei_status fsei_plan_set_precision(fsei_plan* plan, int precision, double rtol, int max_iter);

/* Bytes of device workspace the plan needs in its current precision mode. */
fsei_status fsei_plan_workspace_size(const fsei_plan* plan, size_t* bytes);

/* Hand the plan a device buffer of at least fsei_plan_workspace_size bytes,
 * 256-byte aligned.  Uploads the metric, eigenvalue and twiddle tables with a
 * synchronous copy, and on the first call creates the plan's side stream and
 * two events on the current device (see Execution above).  The buffer stays
 * owned by the caller and must outlive its use by the plan. */
fsei_status fsei_plan_set_workspace(fsei_plan* plan, void* device_ptr, size_t bytes);

/* Stream (a hipStream_t passed as void*) on which all work is enqueued. NULL =
 * the null stream. */
fsei_status fsei_plan_set_stream(fsei_plan* plan, void* hip_stream);

/* Poisson solve p = L^+ f (double I/O; FP64 or FP32_REFINE plans).
 *   f : device, (nz,ny,nx) doubles, read only
 *   p : device, (nz,ny,nx) doubles, written; may alias f
 *   info : optional (host); when given the call waits for the stream. */
fsei_status fsei_poisson_solve(fsei_plan* plan, const double* f, double* p, fsei_info* info);

/* Projection (double I/O; FP64 or FP32_REFINE plans).
 *   u, v, w : device, in: provisional velocity u*, out: projected velocity
 *   p       : device, out: pressure (V-mean zero); may be NULL
 *   dt      : time step (> 0, finite)
 *   info    : optional (host); when given the call waits for the stream. */
fsei_status fsei_project(fsei_plan* plan, double* u, double* v, double* w, double* p, double dt,
                         fsei_info* info);

/* Allocation-free projection, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same operation, arguments, precision modes and results
 * as fsei_project (the same kernels), but the workspace is the library's own
 * static device array of fsei_project_noalloc_max_bytes() bytes (128 MiB),
 * one per GPU, held until the process ends; no workspace needs to be set on
 * the plan and none is used.  The call allocates nothing (no hipMalloc, no
 * library allocation); it copies the plan's tables into the array (host to
 * device, on the plan's stream) and clears its scalars with a kernel.
 *   Limit: fsei_plan_workspace_size(plan) must not exceed
 *   fsei_project_noalloc_max_bytes(), else FSEI_ERR_SCRATCH before any work
 *   (FP64: about 16 M cells; FP32_REFINE: about 5 M cells).
 *   Sharing: all calls on one GPU use the same array, which keeps the last
 *   call's contents; calls that overlap on one GPU (two streams, two threads)
 *   race and give wrong results.  Serialise them. */
fsei_status fsei_project_noalloc(fsei_plan* plan, double* u, double* v, double* w, double* p, double dt,
                                 fsei_info* info);

/* Size in bytes of the static scratch of fsei_project_noalloc. */
size_t fsei_project_noalloc_max_bytes(void);

/* Adjoint of fsei_project with respect to u* (double I/O; FP64 or
 * FP32_REFINE plans, computed in FP64):
 *   g_u* = P^T g_u + (1/dt) D^T (L^+)^T g_p,  P = I - G L^+ D,
 * evaluated as transposed stencils with the stretched-grid metric weights, the
 * transposed per-mode tridiagonal and the transforms in reverse order.
 *   gu, gv, gw : device, in: dLoss/du, out: dLoss/du*
 *   gp         : device, dLoss/dp (read only) or NULL
 *   dt         : the time step of the forward call. */
fsei_status fsei_project_backward(fsei_plan* plan, double* gu, double* gv, double* gw, const double* gp,
                                  double dt);

/* FP32 variants (FSEI_PREC_FP32 plans), same conventions with float fields. */
fsei_status fsei_project_f32(fsei_plan* plan, float* u, float* v, float* w, float* p, float dt);
fsei_status fsei_project_backward_f32(fsei_plan* plan, float* gu, float* gv, float* gw, const float* gp,
                                      float dt);

/* Implicit viscous step of one velocity component (paper, Sec. 2.1, eq.
 * NSdiscr0: Crank-Nicolson for the viscous term; Sec. 3: the 3-D operator is
 * approximately factorised into one tridiagonal operator per direction,
 * inverted with Thomas' algorithm and a Sherman-Morrison correction in the
 * periodic directions).  Solves, in place,
 *
 *     (I - beta L_x)(I - beta L_y)(I - beta L_z) dq = rhs,
 *
 * x factor first, then y, then z.  L_d is the staggered three-point second
 * difference of the component along d: along its own axis (u along x, v
 * along y, w along z) the values are faces, a wall face is Dirichlet zero
 * (the stored wall face is ignored on input and written 0, the opposite wall
 * face is not stored); along the other axes the values are cell centres and
 * a wall is no-slip through a mirrored ghost value; z is stretched (zc of
 * the plan) and always walled; x and y use the plan's boundary types.
 *   component : 0 (u), 1 (v), 2 (w)
 *   q         : device, (nz, ny, nx) FP64; in: rhs, out: dq
 *   beta      : > 0, finite (dt / (2 Re) for Crank-Nicolson)
 * Needs the plan's workspace (it holds the line tables) and nx, ny, nz <=
 * 1024 (FSEI_ERR_SIZE otherwise); works with plans of any precision.  The
 * first call for a component, and any call with a beta different from that
 * component's previous one, waits for the plan's stream once and uploads
 * new tables; otherwise the call only enqueues three kernels. */
fsei_status fsei_viscous_solve(fsei_plan* plan, int component, double* q, double beta);

/* As fsei_viscous_solve, with the increment added to the velocity in the
 * same pass: u <- u + dq (the provisional velocity u* = u^n + du of the
 * fractional step).  rhs is used as scratch (its contents on return are the
 * x and y stages' intermediate, not dq); u must not alias rhs.  dq is 0 on
 * dead wall faces, so those entries of u keep whatever they held (the
 * projection ignores them on input and writes them 0). */
fsei_status fsei_viscous_solve_add(fsei_plan* plan, int component, double* rhs, double* u, double beta);

/* Explicit right-hand side of the momentum step (paper, Sec. 2.1, eq.
 * NSdiscr0: Adams-Bashforth for the convective term with weights gamma, rho
 * (3/2, -1/2; 1, 0 for a first step), Crank-Nicolson for the viscous term;
 * the pressure is left to the projection).  Computes, per component,
 *
 *     rhs = dt [ -(gamma N^n + rho N^{n-1}) + (1/Re) Lap u^n ],   N = div(u u),
 *
 * the right-hand side of the implicit viscous step (fsei_viscous_solve), and
 * N^n for the next step.  N is the divergence form on each component's
 * control volume (two-point means in x and y, linear interpolation in the
 * stretched z, no flux through walls); Lap is the operator of
 * fsei_viscous_solve.  Dead wall faces are ignored on input and written 0.
 *   u, v, w    : device, u^n (read only)
 *   nu, nv, nw : device, in: N^{n-1} (not read when rho == 0), out: N^n
 *   ru, rv, rw : device, out: rhs; must not alias u, v, w, nu, nv, nw
 *   dt, re     : > 0, finite;  gamma, rho: finite
 * All fields (nz, ny, nx) FP64.  Needs the plan's workspace (z metrics). */
fsei_status fsei_momentum_rhs(fsei_plan* plan, const double* u, const double* v, const double* w, double* nu,
                              double* nv, double* nw, double* ru, double* rv, double* rw, double dt, double re,
                              double gamma, double rho);

/* Immersed-boundary moving-least-squares transfer between nb Lagrangian
 * markers and one velocity component (paper, Sec. 2.1, eq. interpv, Fig.
 * mls).  Each marker's support is the 3 x 3 x 3 nodes of the component's own
 * staggered lattice around the node nearest to it (shifted inwards at walls,
 * wrapped across periodic boundaries); the transfer operators are
 * moving-least-squares on the linear basis [1, x, y, z] with the weight
 * exp(-(dx/Dx)^2 - (dy/Dy)^2 - (dz/Hz)^2), Hz the z extent of the middle
 * node's control volume.  They reproduce linear fields exactly.
 *   comp  : 0 (u), 1 (v), 2 (w)
 *   xb    : device, (nb, 3) marker positions x, y, z (any value gives an
 *           in-grid support; positions outside the domain get the nearest one)
 * fsei_ib_interpolate: ub[b] = sum_k phi_k(x_b) field[k]
 *   field : device (nz, ny, nx) FP64, read;  ub: device (nb) FP64, written
 * fsei_ib_spread: field[k] += sum_b phi_k(x_b) fb[b] dvb[b] / V_k, V_k the
 *   node's control volume (dx dy dz_k; dx dy h_k for w): the volume-weighted
 *   transpose of interpolation.  Atomic FP64 additions, so the summation
 *   order (and the last bits) may differ from call to call.
 *   field : device, accumulated;  fb, dvb: device (nb) marker values, volumes
 * nb >= 0 (0: nothing to do); nx, ny, nz >= 3 (FSEI_ERR_SIZE otherwise). */
fsei_status fsei_ib_interpolate(fsei_plan* plan, int comp, const double* field, const double* xb, long nb,
                                double* ub);
fsei_status fsei_ib_spread(fsei_plan* plan, int comp, double* field, const double* xb, const double* fb,
                           const double* dvb, long nb);

/* Per-kernel timing with HIP events on the plan's stream (for measurement).
 * enable != 0 records an event pair around every launch from now on;
 * fsei_plan_reset_timing clears the accumulators. */
fsei_status fsei_plan_set_timing(fsei_plan* plan, int enable);
fsei_status fsei_plan_reset_timing(fsei_plan* plan);

/* Read the accumulated timing of kernel slot `slot` (0 <= slot < FSEI_NUM_KERNEL_SLOTS):
 * total milliseconds and launch count (waits for the stream).  name receives
 * a static string naming the slot's kernel. */
#define FSEI_NUM_KERNEL_SLOTS 22
fsei_status fsei_plan_kernel_time(fsei_plan* plan, int slot, double* total_ms, long* launches,
                                  const char** name);

/* Static description of a status code. */
const char* fsei_status_string(fsei_status status);

#ifdef __cplusplus
}
#endif

#endif /* FSEI_H */
