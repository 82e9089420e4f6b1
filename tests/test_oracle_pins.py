"""Pins of the FP64 oracle against things other than itself (CPU only).

Each test names what fixes the expected value: a library routine for a
special case, the finite-volume definition assembled by loops, exact rational
arithmetic, a closed form, or an invariant of the mathematics.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.fft
import scipy.sparse
import scipy.sparse.linalg

import oracle
from oracle import PERIODIC, WALL, Grid
from paper_2103_15187_amd import workloads as W
import _bruteforce as bf

BCS = [(WALL, WALL), (PERIODIC, WALL), (WALL, PERIODIC), (PERIODIC, PERIODIC)]


def grid_of(spec):
    return Grid(spec.nx, spec.ny, spec.nz, spec.bcx, spec.bcy, spec.dx, spec.dy, spec.zc())


# --------------------------------------------------------------------------
# transforms: special cases that reduce to library routines
# --------------------------------------------------------------------------
# rounding bar for a length-n dot product of unit-size entries with x
def _dot_bar(x):
    return 8 * np.finfo(np.float64).eps * np.abs(x).sum()


@pytest.mark.parametrize("n", [2, 3, 4, 6, 8, 12, 16, 24, 64, 96, 512, 768, 1024])
def test_dct_matrix_is_library_dct2(n):
    x = W.rng(n).standard_normal(n)
    M = oracle.transform_matrix(n, WALL)
    # scipy's unnormalised DCT-II carries a factor 2
    np.testing.assert_allclose(M @ x, scipy.fft.dct(x, type=2) / 2, rtol=0, atol=_dot_bar(x))


@pytest.mark.parametrize("n", [2, 3, 4, 6, 8, 9, 12, 16, 24, 64, 96, 512, 768, 1024])
def test_halfcomplex_matrix_is_library_rfft(n):
    x = W.rng(n + 100).standard_normal(n)
    M = oracle.transform_matrix(n, PERIODIC)
    X = np.fft.rfft(x)
    y = M @ x
    bar = _dot_bar(x)
    for q in range(n // 2 + 1):
        assert abs(y[q] - X[q].real) < bar
    for m in range(1, (n + 1) // 2):
        assert abs(y[n - m] - X[m].imag) < bar


@pytest.mark.parametrize("n,bc", [(n, bc) for n in (2, 3, 5, 8, 12, 16) for bc in (WALL, PERIODIC)])
def test_eigenvalues_diagonalise_1d_stencil(n, bc):
    """M T M^{-1} = diag(lambda) where T is the 1-D second difference built
    from its definition (zero-flux or periodic ends)."""
    d = 0.37
    T = bf.second_difference_matrix(n, d, bc)
    M = oracle.transform_matrix(n, bc)
    D = M @ T @ np.linalg.inv(M)
    lam = oracle.eigenvalues(n, d, bc)
    scale = np.abs(T).max()
    np.testing.assert_allclose(D, np.diag(lam), rtol=0, atol=1e-12 * scale)


# --------------------------------------------------------------------------
# stencils: definition by loops, closed forms, summation by parts
# --------------------------------------------------------------------------
@pytest.mark.parametrize("bc", BCS)
def test_divergence_matches_loop_definition(bc):
    s = W.small_spec(5, 4, 6, bc[0], bc[1], stretch=2.0)
    g = grid_of(s)
    u, v, w = W.random_velocity(s, 11)
    ref = bf.divergence_loops(u, v, w, s.bcx, s.bcy, s.dx, s.dy, s.zc())
    np.testing.assert_allclose(oracle.divergence(u, v, w, g), ref, rtol=1e-14, atol=1e-12)


def test_divergence_of_linear_field_closed_form():
    """u = a x, v = b y, w = c z on active faces (walls at 0 carry 0 anyway);
    interior cells have div = a + b + c exactly."""
    s = W.small_spec(6, 5, 7, WALL, WALL, stretch=1.8)
    g = grid_of(s)
    x = np.arange(s.nx) * s.dx
    y = np.arange(s.ny) * s.dy
    z = s.zc()[:-1]
    u = np.broadcast_to(2.0 * x[None, None, :], s.shape).copy()
    v = np.broadcast_to(-3.0 * y[None, :, None], s.shape).copy()
    w = np.broadcast_to(0.5 * z[:, None, None], s.shape).copy()
    d = oracle.divergence(u, v, w, g)
    inner = d[:-1, :-1, :-1]
    np.testing.assert_allclose(inner, (2.0 - 3.0 + 0.5) * np.ones_like(inner), atol=1e-12)


def test_gradient_of_linear_pressure_closed_form():
    s = W.small_spec(6, 5, 7, PERIODIC, WALL, stretch=2.2)
    g = grid_of(s)
    zc = s.zc()
    zm = 0.5 * (zc[1:] + zc[:-1])
    y = (np.arange(s.ny) + 0.5) * s.dy
    p = 4.0 * y[None, :, None] - 7.0 * zm[:, None, None] + np.zeros(s.shape)
    gx, gy, gz = oracle.gradient(p, g)
    np.testing.assert_allclose(gx, 0.0, atol=1e-12)
    np.testing.assert_allclose(gy[:, 1:, :], 4.0, atol=1e-12)
    np.testing.assert_allclose(gy[:, 0, :], 0.0)       # wall face
    np.testing.assert_allclose(gz[1:], -7.0, atol=1e-12)
    np.testing.assert_allclose(gz[0], 0.0)


@pytest.mark.parametrize("bc", BCS)
def test_summation_by_parts(bc):
    """<D u, q>_V = -<u, G q>_W for every u with zero wall flux."""
    s = W.small_spec(5, 6, 7, bc[0], bc[1], stretch=2.0)
    g = grid_of(s)
    u, v, w = W.random_velocity(s, 5)
    q = W.rng(6).standard_normal(s.shape)
    lhs = (g.cell_volume() * oracle.divergence(u, v, w, g) * q).sum()
    wu, wv, ww = g.face_weights()
    gx, gy, gz = oracle.gradient(q, g)
    rhs = -(wu * u * gx + wv * v * gy + ww * w * gz).sum()
    assert abs(lhs - rhs) < 1e-13 * (abs(lhs) + np.abs(u).sum())


@pytest.mark.parametrize("bc", BCS)
def test_solvability_volume_weighted_divergence_vanishes(bc):
    s = W.small_spec(8, 6, 9, bc[0], bc[1], stretch=2.5)
    g = grid_of(s)
    u, v, w = W.random_velocity(s, 9)
    f = oracle.divergence(u, v, w, g)
    V = g.cell_volume()
    assert abs((V * f).sum()) <= 1e-15 * (V * np.abs(f)).sum() * 10


@pytest.mark.parametrize("bc", BCS)
def test_laplacian_matches_flux_assembly(bc):
    s = W.small_spec(4, 5, 6, bc[0], bc[1], stretch=2.0)
    g = grid_of(s)
    L = bf.dense_laplacian(s.nx, s.ny, s.nz, s.bcx, s.bcy, s.dx, s.dy, s.zc())
    p = W.rng(4).standard_normal(s.shape)
    np.testing.assert_allclose(oracle.laplacian(p, g).ravel(), L @ p.ravel(), rtol=1e-13, atol=1e-10)


@pytest.mark.parametrize("cfg", ["C3", "C5"])
def test_z_coefficients_exact_on_the_workload_grids(cfg):
    """The face coordinates of the tanh-stretched workload grids are binary
    fractions, so Fractions give the exact metric: dz_k = zc_{k+1} - zc_k,
    zm_k = (zc_k + zc_{k+1}) / 2, h_k = zm_k - zm_{k-1}, a_k = 1/(dz_k h_k),
    c_k = 1/(dz_k h_{k+1}) (finite-volume definition, Appendix-style
    loops).  The oracle's FP64 coefficients must be within a few rounding
    steps of these (four operations: 4 ulp)."""
    s = W.CONFIGS[cfg]
    zc = s.zc()
    g = Grid(4, 4, s.nz, WALL, WALL, 1.0, 1.0, zc)
    a, c = oracle.z_coefficients(g)
    zf = [Fraction(float(z)) for z in zc]
    dz = [zf[k + 1] - zf[k] for k in range(s.nz)]
    zm = [(zf[k] + zf[k + 1]) / 2 for k in range(s.nz)]
    ulp = np.finfo(np.float64).eps
    worst = 0.0
    for k in range(s.nz):
        ea = 1 / (dz[k] * (zm[k] - zm[k - 1])) if k >= 1 else Fraction(0)
        ec = 1 / (dz[k] * (zm[k + 1] - zm[k])) if k + 1 < s.nz else Fraction(0)
        for got, ex in ((a[k], ea), (c[k], ec)):
            if ex == 0:
                assert got == 0.0
            else:
                worst = max(worst, abs(float((Fraction(float(got)) - ex) / ex)))
    assert worst <= 4 * ulp, worst


@pytest.mark.parametrize("bc", [(WALL, WALL), (PERIODIC, WALL)])
def test_rel_residual_matches_dense_definition(bc):
    """rel_residual = ||(f - mean_V f) - L p|| / ||f - mean_V f|| with L the
    loop-built flux assembly and the volume-weighted mean of the brute-force
    cell volumes (stretched z: the plain mean differs)."""
    s = W.small_spec(5, 4, 7, bc[0], bc[1], lx=1.3, ly=0.8, lz=2.0, stretch=2.5)
    g = grid_of(s)
    r = W.rng(41)
    f = r.standard_normal(s.shape) + 0.3
    p = r.standard_normal(s.shape)
    L = bf.dense_laplacian(s.nx, s.ny, s.nz, s.bcx, s.bcy, s.dx, s.dy, s.zc())
    V = bf.cell_volumes(s.nx, s.ny, s.nz, s.dx, s.dy, s.zc())
    fc = f.ravel() - (V * f.ravel()).sum() / V.sum()
    ref = np.linalg.norm(fc - L @ p.ravel()) / np.linalg.norm(fc)
    got = oracle.rel_residual(f, p, g)
    assert abs(got - ref) <= 1e-13 * ref
    # the exact solution has (rounding-level) zero residual
    ps = oracle.poisson_solve(f, g)
    assert oracle.rel_residual(f, ps, g) < 1e-13


# --------------------------------------------------------------------------
# the solve: brute force on tiny grids, exact arithmetic, iterative solver
# --------------------------------------------------------------------------
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("dims", [(4, 6, 8), (8, 8, 8), (3, 2, 5), (6, 3, 4)])
def test_solve_matches_bordered_dense_lu(bc, dims):
    nx, ny, nz = dims
    s = W.small_spec(nx, ny, nz, bc[0], bc[1], lx=1.3, ly=0.7, lz=2.0, stretch=2.0)
    g = grid_of(s)
    f = W.rng(nx * 100 + ny * 10 + nz).standard_normal(s.shape)   # not compatible on purpose
    L = bf.dense_laplacian(nx, ny, nz, s.bcx, s.bcy, s.dx, s.dy, s.zc())
    V = bf.cell_volumes(nx, ny, nz, s.dx, s.dy, s.zc())
    p_ref, mu = bf.bordered_solve(L, V, f.ravel())
    p, info = oracle.poisson_solve(f, g, return_info=True)
    scale = np.abs(p_ref).max()
    np.testing.assert_allclose(p.ravel(), p_ref, rtol=0, atol=1e-13 * scale * 10)
    assert abs(info["rhs_vmean_removed"] - mu) < 1e-13 * (1 + abs(mu))


@pytest.mark.parametrize("bc", [(WALL, WALL), (PERIODIC, WALL), (PERIODIC, PERIODIC)])
def test_solve_matches_exact_rational_solution(bc):
    """Exact rational Gauss-Jordan on the bordered system (2 x 3 x 4 cells,
    rational non-uniform z faces) gives p exactly; the FP64 oracle must agree
    to rounding."""
    nx, ny, nz = 2, 3, 4
    dx, dy = Fraction(1, 2), Fraction(1, 3)
    zc = [Fraction(0), Fraction(1, 10), Fraction(1, 2), Fraction(7, 5), Fraction(3, 2)]
    fr = [Fraction(((7 * c) % 11) - 5, 3) for c in range(nx * ny * nz)]
    p_exact, mu = bf.exact_bordered_solve(nx, ny, nz, bc[0], bc[1], dx, dy, zc, fr)
    g = Grid(nx, ny, nz, bc[0], bc[1], float(dx), float(dy), np.array([float(z) for z in zc]))
    f = np.array([float(x) for x in fr]).reshape(nz, ny, nx)
    p, info = oracle.poisson_solve(f, g, return_info=True)
    pe = np.array([float(x) for x in p_exact])
    np.testing.assert_allclose(p.ravel(), pe, rtol=0, atol=1e-13 * np.abs(pe).max())
    assert abs(info["rhs_vmean_removed"] - float(mu)) < 1e-14


def test_solve_matches_conjugate_gradient():
    """Independent iterative solver (CG on the symmetric positive form
    -V L restricted to V-mean-zero fields) on a 24 x 20 x 28 stretched grid."""
    s = W.small_spec(24, 20, 28, PERIODIC, WALL, lx=2.0, ly=1.5, lz=3.0, stretch=2.0)
    g = grid_of(s)
    rows, cols, vals = zip(*bf.laplacian_entries(s.nx, s.ny, s.nz, s.bcx, s.bcy, s.dx, s.dy, list(s.zc())))
    n = s.ncells
    L = scipy.sparse.csr_matrix((vals, (rows, cols)), shape=(n, n))
    V = bf.cell_volumes(s.nx, s.ny, s.nz, s.dx, s.dy, s.zc())
    f = W.rng(77).standard_normal(n)
    f -= (V * f).sum() / V.sum()
    A = -(scipy.sparse.diags(V) @ L)
    b = -(V * f)
    x, info = scipy.sparse.linalg.cg(A, b, rtol=1e-14, atol=0.0, maxiter=20000)
    assert info == 0
    x -= (V * x).sum() / V.sum()
    p = oracle.poisson_solve(f.reshape(s.shape), g).ravel()
    assert np.linalg.norm(p - x) / np.linalg.norm(x) < 1e-10


def test_eigenfunction_recovery_uniform_z():
    """On a uniform z grid the product X_m(i) Y_n(j) Z_l(k) of 1-D stencil
    eigenvectors (taken numerically from the loop-built 1-D matrices) is an
    eigenfunction of L; the solve must return it divided by the eigenvalue."""
    nx, ny, nz = 8, 6, 10
    s = W.small_spec(nx, ny, nz, PERIODIC, WALL, lx=1.0, ly=0.9, lz=1.3, stretch=0.0)
    g = grid_of(s)
    vecs = []
    for n, d, bc in ((nx, s.dx, PERIODIC), (ny, s.dy, WALL), (nz, 1.3 / nz, WALL)):
        T = bf.second_difference_matrix(n, d, bc)
        lam, V = np.linalg.eigh(T)
        vecs.append((lam, V))
    rng = W.rng(3)
    for _ in range(6):
        a, b, c = (int(rng.integers(0, n)) for n in (nx, ny, nz))
        if a == b == c == 0:
            continue
        lam = vecs[0][0][a] + vecs[1][0][b] + vecs[2][0][c]
        if abs(lam) < 1e-9:
            continue
        ph = (vecs[2][1][:, c][:, None, None] * vecs[1][1][:, b][None, :, None]
              * vecs[0][1][:, a][None, None, :])
        p = oracle.poisson_solve(lam * ph, g)
        pe = ph - oracle.vmean(ph, g)
        np.testing.assert_allclose(p, pe, atol=1e-13 * np.abs(pe).max() * 10)


def test_manufactured_random_pressure_stretched():
    """f = L p* (flux assembly) for random p*; the solve returns p* minus its
    V-mean (C2-shaped boundary conditions, strong stretching)."""
    s = W.small_spec(12, 10, 16, PERIODIC, WALL, lx=4.0, ly=4.0, lz=6.5, stretch=2.5)
    g = grid_of(s)
    pst = W.rng(12).standard_normal(s.shape)
    L = bf.dense_laplacian(s.nx, s.ny, s.nz, s.bcx, s.bcy, s.dx, s.dy, s.zc())
    f = (L @ pst.ravel()).reshape(s.shape)
    p = oracle.poisson_solve(f, g)
    pe = pst - oracle.vmean(pst, g)
    assert np.linalg.norm(p - pe) / np.linalg.norm(pe) < 1e-12


def test_zero_mode_prefix_sum_matches_dense():
    s = W.small_spec(1, 1, 9, WALL, WALL, stretch=2.0)
    g = grid_of(s)
    f = W.rng(9).standard_normal(s.nz)
    L = bf.dense_laplacian(1, 1, s.nz, WALL, WALL, 1.0, 1.0, s.zc())
    V = np.diff(s.zc())
    pref, mu = bf.bordered_solve(L, V, f)
    p, mean = oracle.zero_mode_solve(f, g)
    np.testing.assert_allclose(p, pref, atol=1e-13 * np.abs(pref).max())
    assert abs(mean - mu) < 1e-14


# --------------------------------------------------------------------------
# projection: invariants of the discrete mathematics
# --------------------------------------------------------------------------
@pytest.mark.parametrize("bc", BCS)
def test_projection_invariants(bc):
    s = W.small_spec(10, 8, 12, bc[0], bc[1], lx=4.0, ly=4.0, lz=6.5, stretch=2.5)
    g = grid_of(s)
    u, v, w = W.random_velocity(s, 21)
    un, vn, wn, p = oracle.project(u, v, w, g, dt=0.3)
    div = oracle.divergence(un, vn, wn, g)
    assert np.abs(div).max() < 1e-12 * np.abs(oracle.divergence(u, v, w, g)).max()
    assert abs(oracle.vmean(p, g)) < 1e-14 * np.abs(p).max()
    # idempotent
    u2, v2, w2, p2 = oracle.project(un, vn, wn, g)
    for a, b in ((u2, un), (v2, vn), (w2, wn)):
        np.testing.assert_allclose(a, b, atol=1e-12)
    # W-orthogonal decomposition and norm decrease
    wu, wv, ww = g.face_weights()
    cross = (wu * (u - un) * un + wv * (v - vn) * vn + ww * (w - wn) * wn).sum()
    nrm = (wu * un * un + wv * vn * vn + ww * wn * wn).sum()
    nrm0 = (wu * u * u + wv * v * v + ww * w * w).sum()
    assert abs(cross) < 1e-12 * nrm0
    assert nrm <= nrm0
    # dead faces are written zero
    mu, mv, mw = W.dead_face_masks(s)
    assert not un[mu].any() and not vn[mv].any() and not wn[mw].any()


def test_projection_rank():
    """rank P = #active faces - (N - 1)."""
    s = W.small_spec(3, 4, 5, PERIODIC, WALL, stretch=2.0)
    g = grid_of(s)
    mu, mv, mw = g.active_masks()
    act = np.concatenate([mu.ravel(), mv.ravel(), mw.ravel()])
    n = act.size
    cols = []
    for idx in np.flatnonzero(act):
        e = np.zeros(n)
        e[idx] = 1.0
        u, v, w = (e[i * s.ncells:(i + 1) * s.ncells].reshape(s.shape) for i in range(3))
        un, vn, wn, _ = oracle.project(u, v, w, g)
        cols.append(np.concatenate([un.ravel(), vn.ravel(), wn.ravel()])[act])
    P = np.array(cols).T
    assert np.linalg.matrix_rank(P, tol=1e-9) == act.sum() - (s.ncells - 1)


# --------------------------------------------------------------------------
# adjoint: brute-force transpose of the dense maps
# --------------------------------------------------------------------------
@pytest.mark.parametrize("bc", [(PERIODIC, WALL), (WALL, WALL), (WALL, PERIODIC)])
def test_adjoint_is_dense_transpose(bc):
    s = W.small_spec(3, 4, 5, bc[0], bc[1], stretch=2.0)
    g = grid_of(s)
    dt = 0.7
    mu, mv, mw = g.active_masks()
    act = np.concatenate([mu.ravel(), mv.ravel(), mw.ravel()])
    nf = act.size
    N = s.ncells
    P = np.zeros((nf, nf))
    Q = np.zeros((N, nf))
    for idx in np.flatnonzero(act):
        e = np.zeros(nf)
        e[idx] = 1.0
        u, v, w = (e[i * N:(i + 1) * N].reshape(s.shape) for i in range(3))
        un, vn, wn, p = oracle.project(u, v, w, g, dt=dt)
        P[:, idx] = np.concatenate([un.ravel(), vn.ravel(), wn.ravel()])
        Q[:, idx] = p.ravel()
    r = W.rng(8)
    gvec = r.standard_normal(nf) * act
    gp = r.standard_normal(N)
    ref = P.T @ gvec + Q.T @ gp
    gu, gv, gw = (gvec[i * N:(i + 1) * N].reshape(s.shape) for i in range(3))
    ou, ov, ow = oracle.project_adjoint(gu, gv, gw, gp.reshape(s.shape), g, dt=dt)
    out = np.concatenate([ou.ravel(), ov.ravel(), ow.ravel()])
    np.testing.assert_allclose(out, ref * act, atol=1e-12 * np.abs(ref).max())


# --------------------------------------------------------------------------
# floating-point floor: FP64 against long double
# --------------------------------------------------------------------------
@pytest.mark.skipif(np.finfo(np.longdouble).eps >= np.finfo(np.float64).eps,
                    reason="long double is not wider than double here")
def test_fp64_vs_long_double_floor():
    s = W.small_spec(16, 12, 20, PERIODIC, WALL, lx=4.0, ly=4.0, lz=6.5, stretch=2.5)
    g = grid_of(s)
    f = W.rng(31).standard_normal(s.shape)
    p64 = oracle.poisson_solve(f, g)
    pld = oracle.poisson_solve(f.astype(np.longdouble), g, dtype=np.longdouble)
    err = float(np.linalg.norm((p64 - pld).astype(np.float64)) / np.linalg.norm(pld.astype(np.float64)))
    assert err < 1e-13


@pytest.mark.skipif(np.finfo(np.longdouble).eps >= np.finfo(np.float64).eps,
                    reason="long double is not wider than double here")
@pytest.mark.parametrize("n,bc", [(n, bc) for n in (2, 3, 4, 5, 6, 8, 9, 12, 16, 27) for bc in (WALL, PERIODIC)])
def test_closed_form_inverse_in_long_double(n, bc):
    """The long-double variant inverts the transforms by M^T diag(1/||row||^2)
    (rows mutually orthogonal): against Gaussian elimination with partial
    pivoting in long double, and M^-1 M = I to long-double rounding."""
    M = oracle.transform_matrix(n, bc, np.longdouble)
    inv = oracle.inverse_closed_form(M)
    eye = np.eye(n, dtype=np.longdouble)
    from oracle.fsei_oracle import _ld_solve
    elim = _ld_solve(M, eye.copy())
    eps = np.finfo(np.longdouble).eps
    assert np.abs(inv @ M - eye).max() < 64 * n * eps
    assert np.abs(inv - elim).max() < 64 * n * eps * np.abs(elim).max()
    # the FP64 path's solve agrees with it too
    inv64 = np.linalg.solve(M.astype(np.float64), np.eye(n))
    assert np.abs(inv64 - inv.astype(np.float64)).max() < 64 * n * np.finfo(np.float64).eps
