"""Pins of the viscous-step oracle (CPU only).

Each test names what fixes the expected value: the closed-form eigenpairs of
the three-point second difference under each boundary treatment (Fourier
modes for periodic lines, the sine series of the Dirichlet face lines and of
the mirrored-ghost centre lines), the reduction of the stretched z operators
to those uniform ones when the spacing is uniform, the weighted symmetry of
the stretched operators (a finite-volume operator is symmetric in the
volume-weighted inner product), and a dense solve of the full 3-D factorised
operator assembled by Kronecker products.
"""
import numpy as np
import pytest

from oracle import PERIODIC, WALL, Grid
from oracle import viscous as V
from paper_2103_15187_amd import workloads as W


def grid(nx, ny, nz, bcx=WALL, bcy=WALL, stretch=2.0, lx=1.3, ly=0.9, lz=1.7):
    zc = W.tanh_faces(nz, lz, stretch) if stretch > 0 else np.linspace(0.0, lz, nz + 1)
    return Grid(nx, ny, nz, bcx, bcy, lx / nx, ly / ny, zc)


def _line_solve(g, comp, d, beta, line):
    M = V.helmholtz_factor(g, comp, d, beta)
    return np.linalg.solve(M, line)


@pytest.mark.parametrize("n", [3, 8, 12, 17])
@pytest.mark.parametrize("comp", [0, 1, 2])
def test_periodic_fourier_modes(n, comp):
    """Periodic x line: cos(2 pi m i / n + phi) is an eigenvector of the cyclic
    second difference with eigenvalue -4 sin^2(pi m / n) / dx^2, for face and
    centre values alike."""
    g = grid(n, 4, 4, bcx=PERIODIC)
    beta = 0.3 * g.dx**2
    i = np.arange(n)
    for m in range(n):
        q = np.cos(2 * np.pi * m * i / n + 0.4)
        lam = -4.0 * np.sin(np.pi * m / n) ** 2 / g.dx**2
        np.testing.assert_allclose(_line_solve(g, comp, "x", beta, q), q / (1 - beta * lam), atol=1e-13)


@pytest.mark.parametrize("n", [3, 8, 13])
def test_dirichlet_face_sine_modes(n):
    """Wall-normal component along its own axis (u along x, walls): the live
    faces 1..n-1 with zero walls at faces 0 and n carry sin(pi m i / n),
    eigenvalue -4 sin^2(pi m / 2n) / dx^2."""
    g = grid(n, 4, 4, bcx=WALL)
    beta = 0.7 * g.dx**2
    i = np.arange(n)
    for m in range(1, n):
        q = np.sin(np.pi * m * i / n)
        lam = -4.0 * np.sin(np.pi * m / (2 * n)) ** 2 / g.dx**2
        np.testing.assert_allclose(_line_solve(g, 0, "x", beta, q), q / (1 - beta * lam), atol=1e-13)


@pytest.mark.parametrize("n", [2, 5, 8, 12])
@pytest.mark.parametrize("comp", [0, 2])
def test_mirrored_ghost_sine_modes(n, comp):
    """Tangential component at cell centres along a walled y line: the ghost
    q_-1 = -q_0 (zero velocity on the wall) makes sin(pi m (j + 1/2) / n),
    m = 1..n, the eigenvectors, eigenvalue -4 sin^2(pi m / 2n) / dy^2."""
    g = grid(4, n, 4, bcy=WALL)
    beta = 0.45 * g.dy**2
    j = np.arange(n)
    for m in range(1, n + 1):
        q = np.sin(np.pi * m * (j + 0.5) / n)
        lam = -4.0 * np.sin(np.pi * m / (2 * n)) ** 2 / g.dy**2
        np.testing.assert_allclose(_line_solve(g, comp, "y", beta, q), q / (1 - beta * lam), atol=1e-13)


@pytest.mark.parametrize("nz", [3, 7, 16])
def test_uniform_z_reduces_to_uniform_operators(nz):
    """With uniform z spacing the stretched operators are the uniform ones:
    w (faces) equals the Dirichlet face operator, u and v (centres) the
    mirrored-ghost operator, each built along x of a grid with the same
    spacing."""
    lz = 1.1
    gz = grid(4, 4, nz, stretch=0.0, lz=lz)
    gx = Grid(nz, 4, 4, WALL, WALL, lz / nz, 1.0, np.linspace(0, 1, 5))
    np.testing.assert_allclose(V.second_difference(gz, 2, "z"), V.second_difference(gx, 0, "x"), rtol=1e-12)
    for comp in (0, 1):
        np.testing.assert_allclose(V.second_difference(gz, comp, "z"), V.second_difference(gx, 1, "x"),
                                   rtol=1e-12)


@pytest.mark.parametrize("nz", [4, 9, 24])
def test_stretched_z_weighted_symmetry(nz):
    """Finite-volume form: diag(dz) L is symmetric for centre values and
    diag(h) L is symmetric on the live faces for w; every row of a centre
    operator away from the walls sums to zero (constants are in the kernel
    of the interior stencil)."""
    g = grid(4, 4, nz, stretch=2.5)
    Lc = V.second_difference(g, 0, "z")
    S = g.dz[:, None] * Lc
    np.testing.assert_allclose(S, S.T, rtol=1e-12, atol=1e-12 * np.abs(S).max())
    np.testing.assert_allclose(Lc[1:-1].sum(axis=1), 0.0, atol=1e-9 * np.abs(Lc).max())
    Lw = V.second_difference(g, 2, "z")[1:, 1:]
    Sw = g.h[1:, None] * Lw
    np.testing.assert_allclose(Sw, Sw.T, rtol=1e-12, atol=1e-12 * np.abs(Sw).max())
    # wall rows of the centre operator: the half-cell wall flux 2 q / dz
    assert abs(Lc[0, 0] + 2 / g.dz[0] ** 2 + 1 / (g.h[1] * g.dz[0])) < 1e-9 * abs(Lc[0, 0])


def _kron3(Az, Ay, Ax):
    return np.kron(Az, np.kron(Ay, Ax))


@pytest.mark.parametrize("bcx,bcy", [(WALL, WALL), (PERIODIC, WALL), (WALL, PERIODIC), (PERIODIC, PERIODIC)])
@pytest.mark.parametrize("comp", [0, 1, 2])
def test_solve_matches_dense_kronecker_operator(bcx, bcy, comp):
    """The factorised operator (I - bLx)(I - bLy)(I - bLz) assembled as one
    dense matrix of Kronecker products (C order: x fastest) and solved by LU
    on the live unknowns equals the line-by-line solve."""
    g = grid(5, 4, 6, bcx, bcy, stretch=1.8)
    beta = 0.02
    n = g.nx * g.ny * g.nz
    I = [np.eye(m) for m in (g.nz, g.ny, g.nx)]
    Mx = V.helmholtz_factor(g, comp, "x", beta)
    My = V.helmholtz_factor(g, comp, "y", beta)
    Mz = V.helmholtz_factor(g, comp, "z", beta)
    A = _kron3(I[0], I[1], Mx) @ _kron3(I[0], My, I[2]) @ _kron3(Mz, I[1], I[2])
    live = ~V.dead_mask(g, comp).reshape(-1)
    r = W.rng(3 + comp).standard_normal(g.shape)
    x = np.zeros(n)
    x[live] = np.linalg.solve(A[np.ix_(live, live)], r.reshape(-1)[live])
    got = V.viscous_solve(r, g, comp, beta)
    np.testing.assert_allclose(got.reshape(-1), x, rtol=0, atol=1e-12 * np.abs(x).max())
    assert np.all(got[V.dead_mask(g, comp)] == 0)
    # and the factor product applied to the solution reproduces the live input
    back = V.viscous_apply(got, g, comp, beta)
    np.testing.assert_allclose(back[~V.dead_mask(g, comp)], r[~V.dead_mask(g, comp)], atol=1e-12)
