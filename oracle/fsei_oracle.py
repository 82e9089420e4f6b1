"""Plain FP64 CPU oracle for the fractional-step pressure projection.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  The HIP library
(``paper_2103_15187_amd``) never imports it, shares no code, table or constant
generator with it, and fails loudly when its own native code is missing.

What is computed (paper, Sec. 2.1 "Fluid and pressure solver", eqs. NS and
NSdiscr0): the continuity constraint div u = 0 is enforced by a fractional
step in which the pressure acts only as a Lagrange multiplier.  The spatial
discretisation is central second-order finite differences on a staggered
Cartesian mesh (Sec. 2.1).  The time-discrete pressure term is -dt grad p^{n+1}
(eq. NSdiscr0).  The paper does not print the Poisson algorithm; it names FFTW
(Program summary) for the two homogeneous directions (periodic x,y, walls in z,
Sec. 4 and Sec. 5).  This oracle therefore computes the plain discrete object

    f  = D u* / dt                     (cell-centred divergence)
    p  = L^+ f,   L = D G              (V-pseudo-inverse: the V-weighted mean of
                                        f is removed, sum_c V_c p_c = 0)
    u  = u* - dt G p                   (on active faces; dead wall faces = 0)

with the transforms written as dense FP64 matrices (the textbook DCT-II and
real-DFT definitions, no FFT), one Thomas solve per (kx,ky) mode along z, and
the singular (0,0) mode by prefix sums.  Every step is the definition written
out; nothing is blocked, fused or reordered.

Readings of the paper taken here (it is silent on all of them):
  * grid: uniform dx, dy; z faces zc[0..nz] strictly increasing; arrays are
    C-order (nz, ny, nx), x fastest; p at cell centres, u at the low x-face of
    each cell, v at the low y-face, w at the low z-face (w[0] is the bottom
    wall face, the top wall face is not stored);
  * x, y boundary: periodic or wall (zero normal velocity); z: walls;
  * the compact Laplacian L = D G (its eigenvalues in x,y are the modified
    wavenumbers of the 3-point stencil), not a wide centred stencil;
  * zero mode pinned by the volume-weighted mean, sum V p = 0.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

PERIODIC = 0
WALL = 1


# ----------------------------------------------------------------------------
# Grid (Sec. 2.1: staggered Cartesian mesh; z wall-normal, Sec. 4 / Fig. 4)
# ----------------------------------------------------------------------------
@dataclass
class Grid:
    nx: int
    ny: int
    nz: int
    bcx: int
    bcy: int
    dx: float
    dy: float
    zc: np.ndarray                       # nz+1 face coordinates
    dz: np.ndarray = field(init=False)   # cell widths, nz
    zm: np.ndarray = field(init=False)   # cell centres, nz
    h: np.ndarray = field(init=False)    # centre distances, h[k] = zm[k]-zm[k-1], k>=1; h[0] unused

    def __post_init__(self):
        self.zc = np.asarray(self.zc, dtype=np.float64)
        assert self.zc.shape == (self.nz + 1,)
        self.dz, self.h = self.z_metrics(np.float64)
        assert np.all(self.dz > 0), "zc must be strictly increasing"
        self.zm = 0.5 * (self.zc[1:] + self.zc[:-1])

    def z_metrics(self, dtype=np.float64):
        """Cell widths dz_k = zc_{k+1} - zc_k and centre distances
        h_k = zm_k - zm_{k-1}, evaluated in `dtype`.  h_k is written as
        (dz_{k-1} + dz_k) / 2, which equals the difference of the two
        midpoints in exact arithmetic but rounds once from the widths instead
        of cancelling two rounded midpoints (on a strongly stretched grid the
        cancellation costs up to ~5e-12 relative near the walls)."""
        zc = self.zc.astype(dtype)
        dz = np.diff(zc)
        h = np.empty(self.nz, dtype=dtype)
        h[0] = np.nan
        h[1:] = (dz[:-1] + dz[1:]) / 2
        return dz, h

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def cell_volume(self):
        """V_c = dx dy dz_k, broadcast to (nz, ny, nx)."""
        return np.broadcast_to((self.dx * self.dy * self.dz)[:, None, None], self.shape)

    def face_weights(self):
        """W for the u, v, w faces: x- and y-faces dx dy dz_k, z-faces dx dy h_k
        (dead faces get weight 1 so that W^-1 is defined; their values are 0)."""
        wxy = (self.dx * self.dy * self.dz)[:, None, None] * np.ones(self.shape)
        hz = self.h.copy()
        hz[0] = 1.0
        wz = (self.dx * self.dy * hz)[:, None, None] * np.ones(self.shape)
        return wxy, wxy.copy(), wz

    def active_masks(self):
        """Boolean masks of the active u, v, w faces."""
        mu = np.ones(self.shape, dtype=bool)
        mv = np.ones(self.shape, dtype=bool)
        mw = np.ones(self.shape, dtype=bool)
        if self.bcx == WALL:
            mu[:, :, 0] = False
        if self.bcy == WALL:
            mv[:, 0, :] = False
        mw[0, :, :] = False
        return mu, mv, mw


# ----------------------------------------------------------------------------
# Staggered stencils (Sec. 2.1: central second-order FD on a staggered mesh)
# ----------------------------------------------------------------------------
def _faces_hi(a, axis, bc):
    """Value of the face on the high side of each cell along `axis`:
    a[..., i+1]; at the last cell it is the wrapped face 0 (periodic) or the
    wall face, whose normal velocity is 0."""
    hi = np.roll(a, -1, axis=axis)
    if bc == WALL:
        idx = [slice(None)] * 3
        idx[axis] = -1
        hi[tuple(idx)] = 0.0
    return hi


def _zero_dead(u, v, w, g: Grid):
    mu, mv, mw = g.active_masks()
    return np.where(mu, u, 0.0), np.where(mv, v, 0.0), np.where(mw, w, 0.0)


def divergence(u, v, w, g: Grid):
    """(D u)_c = (u_{i+1}-u_i)/dx + (v_{j+1}-v_j)/dy + (w_{k+1}-w_k)/dz_k.
    Dead wall faces are read as zero."""
    u, v, w = _zero_dead(u, v, w, g)
    du = (_faces_hi(u, 2, g.bcx) - u) / g.dx
    dv = (_faces_hi(v, 1, g.bcy) - v) / g.dy
    dw = (_faces_hi(w, 0, WALL) - w) / g.dz[:, None, None]
    return du + dv + dw


def gradient(p, g: Grid):
    """(G p) on faces: (p_i - p_{i-1})/dx, (p_j - p_{j-1})/dy, (p_k - p_{k-1})/h_k
    on active faces, 0 on dead wall faces."""
    gx = (p - np.roll(p, 1, axis=2)) / g.dx
    gy = (p - np.roll(p, 1, axis=1)) / g.dy
    hz = g.h.copy()
    hz[0] = 1.0
    gz = (p - np.roll(p, 1, axis=0)) / hz[:, None, None]
    return _zero_dead(gx, gy, gz, g)


def laplacian(p, g: Grid):
    """L p = D (G p)."""
    return divergence(*gradient(p, g), g)


# ----------------------------------------------------------------------------
# Transforms in the homogeneous directions, as dense matrices (the plain
# definitions; the paper uses FFTW for these, Program summary)
# ----------------------------------------------------------------------------
def transform_matrix(n: int, bc: int, dtype=np.float64) -> np.ndarray:
    """Forward transform matrix M (rows = modes q, columns = points i).

    wall:     M[q, i] = cos(pi q (i + 1/2) / n)               (DCT-II)
    periodic: half-complex real DFT, M[q, i] = cos(2 pi q i / n) for q <= n/2,
              M[n-m, i] = -sin(2 pi m i / n) for 0 < m < n/2 (Im of the DFT).

    The angles are multiples of pi/(2n); the integer multiple is reduced
    modulo one period exactly (integer arithmetic) before the cosine is
    taken, so each entry is accurate to rounding even when q*i is large."""
    i = np.arange(n, dtype=np.int64)
    M = np.empty((n, n), dtype=dtype)
    pi = dtype(np.pi) if dtype is not np.longdouble else np.longdouble("3.14159265358979323846264338327950288")
    if bc == WALL:
        # pi q (2i+1) / (2n): multiple r = q (2i+1) of pi/(2n), period 4n
        for q in range(n):
            r = (q * (2 * i + 1)) % (4 * n)
            M[q] = np.cos(pi * r.astype(dtype) / (2 * n))
    else:
        # 2 pi q i / n: multiple r = q i of 2 pi / n, period n
        for q in range(n // 2 + 1):
            r = (q * i) % n
            M[q] = np.cos(2 * pi * r.astype(dtype) / n)
        for m in range(1, (n + 1) // 2):
            r = (m * i) % n
            M[n - m] = -np.sin(2 * pi * r.astype(dtype) / n)
    return M


def mode_wavenumber(n: int, bc: int) -> np.ndarray:
    """Integer wavenumber m(q) of transform row q."""
    q = np.arange(n)
    return q if bc == WALL else np.minimum(q, n - q)


def eigenvalues(n: int, d: float, bc: int, dtype=np.float64) -> np.ndarray:
    """Eigenvalue of the 3-point second difference (1D part of L) on row q:
    wall -(4/d^2) sin^2(pi m / (2n)); periodic -(4/d^2) sin^2(pi m / n)."""
    m = mode_wavenumber(n, bc).astype(dtype)
    pi = dtype(np.pi) if dtype is not np.longdouble else np.longdouble("3.14159265358979323846264338327950288")
    arg = pi * m / (2 * n) if bc == WALL else pi * m / n
    return -(dtype(4) / (dtype(d) * dtype(d))) * np.sin(arg) ** 2


def _apply_along(M, a, axis):
    """Apply matrix M along `axis` of a 3-D array."""
    return np.moveaxis(np.tensordot(M, a, axes=([1], [axis])), 0, axis)


def _solve_along(M, a, axis):
    """Apply M^{-1} along `axis`: a linear solve with M in FP64; in long
    double the closed-form inverse (numpy's LAPACK path has no long-double
    solver, and elimination in Python loops is O(n^3) per call)."""
    a = np.moveaxis(a, axis, 0)
    shp = a.shape
    if M.dtype != np.longdouble:
        x = np.linalg.solve(M, a.reshape(shp[0], -1))
    else:
        x = inverse_closed_form(M) @ a.reshape(shp[0], -1)
    return np.moveaxis(x.reshape(shp), 0, axis)


def inverse_closed_form(M):
    """M^{-1} = M^T diag(1 / ||row_q||^2) for the transform matrices of
    transform_matrix: their rows are mutually orthogonal (the DCT-II rows,
    and the cosine and sine rows of the real DFT), with squared norms n for
    the constant row and the periodic Nyquist row and n/2 for every other."""
    n = M.shape[0]
    w = np.einsum("qi,qi->q", M, M)
    return M.T * (1 / w)[None, :]


def _ld_solve(M, B):
    """Gaussian elimination with partial pivoting in long double (numpy's
    LAPACK path has no long-double solver); the reference the closed-form
    inverse is pinned against."""
    n = M.shape[0]
    A = M.copy()
    X = B.copy()
    for col in range(n):
        piv = col + int(np.argmax(np.abs(A[col:, col])))
        if piv != col:
            A[[col, piv]] = A[[piv, col]]
            X[[col, piv]] = X[[piv, col]]
        inv = 1 / A[col, col]
        for r in range(col + 1, n):
            fct = A[r, col] * inv
            if fct != 0:
                A[r, col:] -= fct * A[col, col:]
                X[r] -= fct * X[col]
    for col in range(n - 1, -1, -1):
        X[col] = (X[col] - A[col, col + 1:] @ X[col + 1:]) / A[col, col]
    return X


# ----------------------------------------------------------------------------
# z direction: one tridiagonal per (kx,ky) mode
# ----------------------------------------------------------------------------
def z_coefficients(g: Grid, dtype=np.float64):
    """Off-diagonals of the z part of L = D G on cell centres with wall
    (zero-flux) ends: (L_z p)_k = a_k p_{k-1} - (a_k + c_k) p_k + c_k p_{k+1},
    a_k = 1/(dz_k h_k) (k>=1), c_k = 1/(dz_k h_{k+1}) (k<=nz-2)."""
    nz = g.nz
    dz, h = g.z_metrics(dtype)
    a = np.zeros(nz, dtype=dtype)
    c = np.zeros(nz, dtype=dtype)
    a[1:] = 1 / (dz[1:] * h[1:])
    c[:-1] = 1 / (dz[:-1] * h[1:])
    return a, c


def thomas(a, b, c, f):
    """Thomas algorithm for a_k x_{k-1} + b_k x_k + c_k x_{k+1} = f_k along
    axis 0, vectorised over the trailing axes (b and f have the same shape)."""
    n = f.shape[0]
    cp = np.empty_like(f)
    dp = np.empty_like(f)
    cp[0] = c[0] / b[0]
    dp[0] = f[0] / b[0]
    for k in range(1, n):
        den = b[k] - a[k] * cp[k - 1]
        cp[k] = c[k] / den
        dp[k] = (f[k] - a[k] * dp[k - 1]) / den
    x = np.empty_like(f)
    x[n - 1] = dp[n - 1]
    for k in range(n - 2, -1, -1):
        x[k] = dp[k] - cp[k] * x[k + 1]
    return x


def zero_mode_solve(fhat0, g: Grid):
    """(0,0) mode: L_z p = f is singular (zero-flux walls).  Remove the
    dz-weighted mean of f (compatibility), integrate the flux
    F_k = sum_{k'<k} dz_k' f_k', then p_k = p_{k-1} + h_k F_k, and pin
    sum_k dz_k p_k = 0.  Returns (p, removed dz-weighted mean)."""
    dz, h = g.z_metrics(fhat0.dtype)
    lz = dz.sum()
    mean = (dz * fhat0).sum() / lz
    f = fhat0 - mean
    flux = np.zeros(g.nz, dtype=fhat0.dtype)
    flux[1:] = np.cumsum(dz[:-1] * f[:-1])
    p = np.zeros(g.nz, dtype=fhat0.dtype)
    for k in range(1, g.nz):
        p[k] = p[k - 1] + h[k] * flux[k]
    p -= (dz * p).sum() / lz
    return p, mean


# ----------------------------------------------------------------------------
# Poisson solve and projection
# ----------------------------------------------------------------------------
def poisson_solve(f, g: Grid, dtype=np.float64, return_info=False):
    """p = L^+ f: the V-weighted mean of f is removed, L p = f - mean_V(f),
    sum_c V_c p_c = 0.  Transforms along x then y, per-mode tridiagonal along
    z, inverse transforms along y then x."""
    f = np.asarray(f, dtype=dtype)
    Mx = transform_matrix(g.nx, g.bcx, dtype)
    My = transform_matrix(g.ny, g.bcy, dtype)
    fh = _apply_along(My, _apply_along(Mx, f, 2), 1)            # (nz, ny, nx) in modes
    lx = eigenvalues(g.nx, g.dx, g.bcx, dtype)
    ly = eigenvalues(g.ny, g.dy, g.bcy, dtype)
    a, c = z_coefficients(g, dtype)
    # modes flattened to (nz, ny*nx); mode (0,0) is column 0 and singular, so
    # Thomas runs on columns 1.. and (0,0) is solved by prefix sums
    sigma = (ly[:, None] + lx[None, :]).reshape(-1)             # (ny*nx,)
    fhm = fh.reshape(g.nz, -1)
    phm = np.empty_like(fhm)
    b = (-(a + c))[:, None] + sigma[None, 1:]
    phm[:, 1:] = thomas(a, b, c, fhm[:, 1:])
    p00, mean00 = zero_mode_solve(fhm[:, 0], g)
    phm[:, 0] = p00
    ph = phm.reshape(fh.shape)
    p = _solve_along(Mx, _solve_along(My, ph, 1), 2)
    if return_info:
        # mode (0,0) of both transforms is the plain sum over (x,y)
        return p, {"rhs_vmean_removed": float(mean00 / (g.nx * g.ny))}
    return p


def project(u, v, w, g: Grid, dt=1.0, dtype=np.float64):
    """Fractional-step projection: f = D u*/dt, p = L^+ f, u = u* - dt G p.
    Returns (u, v, w, p); dead wall faces are 0 on output."""
    f = divergence(u, v, w, g) / dt
    p = poisson_solve(f, g, dtype)
    gx, gy, gz = gradient(p, g)
    un, vn, wn = _zero_dead(u - dt * gx, v - dt * gy, w - dt * gz, g)
    return un, vn, wn, p


def project_adjoint(gu, gv, gw, gp, g: Grid, dt=1.0, dtype=np.float64):
    """Adjoint of `project` with respect to u*.  With V D = -G^T W
    (summation by parts), P = I - G L^+ D satisfies P^T = W P W^{-1} and
    (L^+)^T = V L^+ V^{-1}, so

        g_u* = W P (W^-1 g_u) - (1/dt) W G L^+ (V^-1 g_p).

    This uses only the oracle's own forward operators (their solves in
    `dtype`)."""
    wu, wv, ww = g.face_weights()
    xu, xv, xw = _zero_dead(gu / wu, gv / wv, gw / ww, g)
    pu, pv, pw, _ = project(xu, xv, xw, g, dt=1.0, dtype=dtype)
    ou, ov, ow = wu * pu, wv * pv, ww * pw
    if gp is not None:
        s = poisson_solve(gp / g.cell_volume(), g, dtype=dtype)
        sx, sy, sz = gradient(s, g)
        ou = ou - wu * sx / dt
        ov = ov - wv * sy / dt
        ow = ow - ww * sz / dt
    return _zero_dead(ou, ov, ow, g)


def vmean(p, g: Grid):
    """Volume-weighted mean sum V p / sum V."""
    V = g.cell_volume()
    return float((V * p).sum() / V.sum())


def rel_residual(f, p, g: Grid):
    """||f - mean_V(f) - L p||_2 / ||f - mean_V(f)||_2 over cells."""
    fc = f - vmean(f, g)
    r = fc - laplacian(p, g)
    return float(np.linalg.norm(r) / np.linalg.norm(fc))
