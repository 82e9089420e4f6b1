"""Pins of the IB-MLS transfer oracle (CPU only).

What fixes the expected values: the defining properties of a linear-basis
moving-least-squares operator (it reproduces every linear field: the operators
sum to 1 and their first moments about the marker vanish), its equivalence
with a weighted least-squares linear fit computed by a library routine
(numpy.linalg.lstsq on the square-root-weighted system), and the volume
weighted transpose relation between spreading and interpolation.
"""
import numpy as np
import pytest

from oracle import PERIODIC, WALL, Grid
from oracle import ibm_oracle as I
from paper_2103_15187_amd import workloads as W

BCS = [(WALL, WALL), (PERIODIC, WALL), (WALL, PERIODIC), (PERIODIC, PERIODIC)]


def grid(bc, nx=16, ny=12, nz=20, stretch=2.0):
    return Grid(nx, ny, nz, bc[0], bc[1], 1.6 / nx, 1.2 / ny, W.tanh_faces(nz, 2.0, stretch))


def markers(g, nb, seed):
    r = W.rng(seed)
    return np.stack([r.uniform(0, g.nx * g.dx, nb), r.uniform(0, g.ny * g.dy, nb), r.uniform(0, g.zc[-1], nb)], 1)


def _volumes_z(g, comp):
    """z extent of each node's control volume, written out here: the cell
    width for u, v (cell centres in z); for w on face k the distance between
    the centres around it, half the first cell at the wall face k = 0."""
    zc = g.zc
    if comp != 2:
        return np.diff(zc)
    zm = 0.5 * (zc[1:] + zc[:-1])
    return np.concatenate([[0.5 * (zc[1] - zc[0])], np.diff(zm)])


def _displacements(g, comp, xb, flat):
    x, y, z = I.node_coords(g, comp)
    kz, rem = np.divmod(flat, g.nx * g.ny)
    jy, ix = np.divmod(rem, g.nx)
    d = np.stack([x[ix] - xb[0], y[jy] - xb[1], z[kz] - xb[2]], 1)
    for a, (per, L) in enumerate(((g.bcx != WALL, g.nx * g.dx), (g.bcy != WALL, g.ny * g.dy))):
        if per:
            d[:, a] -= L * np.round(d[:, a] / L)
    return d


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("comp", [0, 1, 2])
def test_reproduces_linear_fields(bc, comp):
    """sum phi_k = 1 and sum phi_k (x_k - x_b) = 0 (per axis) for every marker,
    near walls and across periodic seams."""
    g = grid(bc)
    for xb in markers(g, 60, 5 + comp):
        flat, phi = I.shape_functions(g, comp, xb)
        d = _displacements(g, comp, xb, flat)
        assert abs(phi.sum() - 1.0) < 1e-13
        np.testing.assert_allclose(phi @ d, 0.0, atol=1e-14)


@pytest.mark.parametrize("comp", [0, 1, 2])
def test_matches_weighted_least_squares_fit(comp):
    """The interpolated value is the intercept of the W-weighted linear fit of
    the 27 support values (library least squares)."""
    g = grid((PERIODIC, WALL))
    u = W.rng(9).standard_normal(g.shape)
    xb = markers(g, 40, 10 + comp)
    got = I.interpolate(u, g, comp, xb)
    for b, x in enumerate(xb):
        flat, _ = I.shape_functions(g, comp, x)
        d = _displacements(g, comp, x, flat)
        hz = _volumes_z(g, comp)[np.divmod(flat, g.nx * g.ny)[0][13]]
        Wk = np.exp(-(d[:, 0] / g.dx) ** 2 - (d[:, 1] / g.dy) ** 2 - (d[:, 2] / hz) ** 2)
        P = np.concatenate([np.ones((27, 1)), d], 1)
        s = np.sqrt(Wk)
        coef, *_ = np.linalg.lstsq(P * s[:, None], u.reshape(-1)[flat] * s, rcond=None)
        assert abs(got[b] - coef[0]) < 1e-12 * max(1.0, abs(coef[0]))


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("comp", [0, 1, 2])
def test_spreading_is_the_volume_weighted_transpose(bc, comp):
    """sum_b dV_b F_b (I u)_b = sum_k V_k (S F)_k u_k for arbitrary u, F."""
    g = grid(bc)
    r = W.rng(20 + comp)
    xb = markers(g, 50, 30 + comp)
    fb = r.standard_normal(50)
    dv = r.uniform(0.5, 1.5, 50) * 1e-3
    u = r.standard_normal(g.shape)
    f = I.spread(g, comp, xb, fb, dv)
    vz = _volumes_z(g, comp)
    lhs = (dv * fb * I.interpolate(u, g, comp, xb)).sum()
    rhs = (f * u * (g.dx * g.dy * vz[:, None, None])).sum()
    assert abs(lhs - rhs) < 1e-13 * (np.abs(dv * fb).sum() * np.abs(u).max())


@pytest.mark.parametrize("comp", [0, 1, 2])
def test_linear_field_on_the_staggered_positions(comp):
    """A linear function sampled where the staggered grid stores component
    comp (u on x faces i dx, v on y faces j dy, w on z faces zc[k], cell
    centres along the other axes; positions written out here, not taken from
    the oracle) is reproduced exactly at any marker: pins the node positions."""
    g = grid((WALL, WALL))
    zc = g.zc
    xs = np.arange(g.nx) * g.dx + (0.0 if comp == 0 else 0.5 * g.dx)
    ys = np.arange(g.ny) * g.dy + (0.0 if comp == 1 else 0.5 * g.dy)
    zs = zc[:-1] if comp == 2 else 0.5 * (zc[1:] + zc[:-1])
    a, bx, by, bz = 0.4, 1.3, -0.6, 2.1
    field = a + bx * xs[None, None, :] + by * ys[None, :, None] + bz * zs[:, None, None]
    xb = markers(g, 80, 60 + comp)
    got = I.interpolate(field, g, comp, xb)
    exact = a + bx * xb[:, 0] + by * xb[:, 1] + bz * xb[:, 2]
    np.testing.assert_allclose(got, exact, rtol=0, atol=1e-12 * np.abs(exact).max())
