"""Plant plausible mistakes in the viscous-step oracle (on the CPU) and check
that its pins catch every one of them."""
import numpy as np
import pytest

import oracle.viscous_oracle as V
import test_viscous_oracle as pins
from oracle import PERIODIC, WALL


def _run_pins():
    checks = [
        lambda: pins.test_periodic_fourier_modes(8, 1),
        lambda: pins.test_periodic_fourier_modes(8, 0),
        lambda: pins.test_dirichlet_face_sine_modes(8),
        lambda: pins.test_mirrored_ghost_sine_modes(8, 0),
        lambda: pins.test_uniform_z_reduces_to_uniform_operators(7),
        lambda: pins.test_stretched_z_weighted_symmetry(9),
        lambda: pins.test_solve_matches_dense_kronecker_operator(PERIODIC, WALL, 2),
        lambda: pins.test_solve_matches_dense_kronecker_operator(WALL, PERIODIC, 0),
    ]
    failed = 0
    for c in checks:
        try:
            c()
        except (AssertionError, ValueError, np.linalg.LinAlgError):
            failed += 1
    return failed


ORIG = V.second_difference


def _mut_ghost_weight(g, comp, direction):
    """no-slip ghost taken as zero-gradient (q_ghost = q) instead of mirrored"""
    L = ORIG(g, comp, direction).copy()
    own = {"x": 0, "y": 1, "z": 2}[direction] == comp
    if direction in ("x", "y") and not own and (g.bcx if direction == "x" else g.bcy) == WALL:
        d = g.dx if direction == "x" else g.dy
        L[0, 0] += 2.0 / d**2
        L[-1, -1] += 2.0 / d**2
    return L


def _mut_z_centre_dz(g, comp, direction):
    """centre z operator with cell widths where the centre distances belong"""
    if direction != "z" or comp == 2:
        return ORIG(g, comp, direction)
    L = ORIG(g, comp, direction).copy()
    n = g.nz
    for k in range(1, n):
        L[k, k - 1] = 1.0 / (g.dz[k - 1] * g.dz[k])
    for k in range(n):
        L[k, k] = -(np.sum(L[k]) - L[k, k]) - (2.0 / g.dz[k] ** 2 if k in (0, n - 1) else 0.0)
    return L


def _mut_z_face_swap(g, comp, direction):
    """face z operator divided by the cell width instead of the centre distance"""
    if direction != "z" or comp != 2:
        return ORIG(g, comp, direction)
    L = ORIG(g, comp, direction).copy()
    for k in range(1, g.nz):
        L[k] *= g.h[k] / g.dz[k]
    return L


def _mut_wall_face_live(g, comp, direction):
    """the wall face along the component's own axis left live"""
    own = {"x": 0, "y": 1, "z": 2}[direction] == comp
    L = ORIG(g, comp, direction).copy()
    if own and direction == "x" and g.bcx == WALL:
        d = g.dx
        L[0, 0] = -2.0 / d**2
        L[0, 1] = L[1, 0] = 1.0 / d**2
    return L


def _mut_no_wrap(g, comp, direction):
    """periodic line without the wrap-around coupling"""
    L = ORIG(g, comp, direction).copy()
    if direction in ("x", "y") and (g.bcx if direction == "x" else g.bcy) == PERIODIC and L.shape[0] > 2:
        L[0, -1] = 0.0
        L[-1, 0] = 0.0
    return L


MUTANTS = {"ghost_weight": _mut_ghost_weight, "z_centre_dz": _mut_z_centre_dz, "z_face_swap": _mut_z_face_swap,
           "wall_face_live": _mut_wall_face_live, "no_wrap": _mut_no_wrap}


def test_unmutated_oracle_passes_the_subset():
    assert _run_pins() == 0


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, monkeypatch):
    monkeypatch.setattr(V, "second_difference", MUTANTS[name])
    assert _run_pins() >= 1, name
