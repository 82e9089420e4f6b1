"""Plant plausible mistakes in the oracle (on the CPU) and check that the pins
catch every one of them.  Each mutant must make at least one pin fail."""
import numpy as np
import pytest

import oracle
import oracle.fsei_oracle as O
import test_oracle_pins as pins
from oracle import PERIODIC, WALL


def _run_pins():
    """Run a representative subset of pins; return the number that failed."""
    checks = [
        lambda: pins.test_dct_matrix_is_library_dct2(8),
        lambda: pins.test_halfcomplex_matrix_is_library_rfft(8),
        lambda: pins.test_eigenvalues_diagonalise_1d_stencil(8, WALL),
        lambda: pins.test_eigenvalues_diagonalise_1d_stencil(8, PERIODIC),
        lambda: pins.test_divergence_matches_loop_definition((PERIODIC, WALL)),
        lambda: pins.test_summation_by_parts((WALL, WALL)),
        lambda: pins.test_solve_matches_bordered_dense_lu((PERIODIC, WALL), (4, 6, 8)),
        lambda: pins.test_solve_matches_bordered_dense_lu((WALL, WALL), (3, 2, 5)),
        lambda: pins.test_projection_invariants((WALL, PERIODIC)),
        lambda: pins.test_adjoint_is_dense_transpose((PERIODIC, WALL)),
        lambda: pins.test_z_coefficients_exact_on_the_workload_grids("C3"),
        lambda: pins.test_rel_residual_matches_dense_definition((WALL, WALL)),
    ]
    failed = 0
    for c in checks:
        try:
            c()
        except (AssertionError, ValueError, FloatingPointError, np.linalg.LinAlgError):
            failed += 1
    return failed


def test_unmutated_oracle_passes_the_subset():
    assert _run_pins() == 0


def _mut_div_uses_h(u, v, w, g):
    u, v, w = O._zero_dead(u, v, w, g)
    hz = g.h.copy()
    hz[0] = g.dz[0]
    du = (O._faces_hi(u, 2, g.bcx) - u) / g.dx
    dv = (O._faces_hi(v, 1, g.bcy) - v) / g.dy
    dw = (O._faces_hi(w, 0, WALL) - w) / hz[:, None, None]
    return du + dv + dw


def _mut_grad_sign(p, g):
    gx, gy, gz = ORIG["gradient"](p, g)
    return gx, -gy, gz


def _mut_eig_wall_arg(n, d, bc, dtype=np.float64):
    m = O.mode_wavenumber(n, bc).astype(dtype)
    return -(4 / d ** 2) * np.sin(np.pi * m / n) ** 2


def _mut_zcoef_index(g, dtype=np.float64):
    a, c = ORIG["z_coefficients"](g, dtype)
    c2 = np.zeros_like(c)
    c2[:-1] = 1 / (g.dz[:-1] * g.h[1:]) * (g.dz[:-1] / g.dz[1:])
    return a, c2


def _mut_thomas_swap(a, b, c, f):
    return ORIG["thomas"](c, b, a, f)


def _mut_zero_mode_no_pin(fhat0, g):
    p, mean = ORIG["zero_mode_solve"](fhat0, g)
    return p + 0.1 * np.abs(p).max(), mean


def _mut_dct_no_half(n, bc, dtype=np.float64):
    if bc != WALL:
        return ORIG["transform_matrix"](n, bc, dtype)
    i = np.arange(n, dtype=dtype)
    return np.array([np.cos(np.pi * q * i / n) for q in range(n)])


def _mut_transform_transposed(n, bc, dtype=np.float64):
    return ORIG["transform_matrix"](n, bc, dtype).T.copy()


def _mut_adjoint_no_weights(gu, gv, gw, gp, g, dt=1.0):
    pu, pv, pw, _ = O.project(gu, gv, gw, g, dt=1.0)
    return pu, pv, pw


def _mut_h_from_midpoints(self, dtype=np.float64):
    zc = self.zc.astype(dtype)
    zm = (zc[1:] + zc[:-1]) / 2
    h = np.empty(self.nz, dtype=dtype)
    h[0] = np.nan
    h[1:] = np.diff(zm)
    return np.diff(zc), h


def _mut_residual_plain_mean(f, p, g):
    fc = f - f.mean()
    r = fc - O.laplacian(p, g)
    return float(np.linalg.norm(r) / np.linalg.norm(fc))


ORIG = {name: getattr(O, name) for name in
        ("divergence", "gradient", "eigenvalues", "z_coefficients", "thomas",
         "zero_mode_solve", "transform_matrix", "project_adjoint", "rel_residual")}

MUTANTS = {
    "divergence z metric uses h": ("divergence", _mut_div_uses_h),
    "gradient sign flipped in y": ("gradient", _mut_grad_sign),
    "wall eigenvalue with periodic argument": ("eigenvalues", _mut_eig_wall_arg),
    "z super-diagonal from the wrong cell": ("z_coefficients", _mut_zcoef_index),
    "tridiagonal operands transposed": ("thomas", _mut_thomas_swap),
    "zero mode not pinned": ("zero_mode_solve", _mut_zero_mode_no_pin),
    "DCT-II without the half-cell shift": ("transform_matrix", _mut_dct_no_half),
    "transform matrix transposed": ("transform_matrix", _mut_transform_transposed),
    "adjoint without metric weights": ("project_adjoint", _mut_adjoint_no_weights),
    "h as the difference of rounded midpoints": ("Grid.z_metrics", _mut_h_from_midpoints),
    "residual centred by the plain mean": ("rel_residual", _mut_residual_plain_mean),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, monkeypatch):
    attr, fn = MUTANTS[name]
    if attr.startswith("Grid."):
        monkeypatch.setattr(O.Grid, attr.split(".")[1], fn)
    else:
        monkeypatch.setattr(O, attr, fn)
        if hasattr(oracle, attr):
            monkeypatch.setattr(oracle, attr, fn)
    with np.errstate(all="ignore"):
        assert _run_pins() >= 1, f"no pin caught the mutant: {name}"
