"""Plant plausible mistakes in the IB-MLS transfer oracle (on the CPU, by
editing a copy of its source) and check that its pins catch each."""
import inspect
import types

import pytest

import oracle.ibm_oracle as I
import test_ibm_oracle as pins
from oracle import PERIODIC, WALL


def _run_pins():
    checks = [
        lambda: pins.test_reproduces_linear_fields((WALL, WALL), 0),
        lambda: pins.test_reproduces_linear_fields((PERIODIC, PERIODIC), 2),
        lambda: pins.test_matches_weighted_least_squares_fit(0),
        lambda: pins.test_matches_weighted_least_squares_fit(2),
        lambda: pins.test_spreading_is_the_volume_weighted_transpose((PERIODIC, WALL), 1),
        lambda: pins.test_spreading_is_the_volume_weighted_transpose((WALL, WALL), 2),
        lambda: pins.test_linear_field_on_the_staggered_positions(0),
        lambda: pins.test_linear_field_on_the_staggered_positions(1),
        lambda: pins.test_linear_field_on_the_staggered_positions(2),
    ]
    failed = 0
    for c in checks:
        try:
            c()
        except (AssertionError, ValueError, IndexError):
            failed += 1
    return failed


# (original text, mutated text): each a plausible slip in the transfer
MUTANTS = {
    "weight_scale_of_an_outer_node": ("hz = node_volumes_z(g, comp)[iz[1]]", "hz = node_volumes_z(g, comp)[iz[0]]"),
    "weight_without_z": ("Wk = np.exp(-(P[:, 1] / g.dx) ** 2 - (P[:, 2] / g.dy) ** 2 - (P[:, 3] / hz) ** 2)",
                         "Wk = np.exp(-(P[:, 1] / g.dx) ** 2 - (P[:, 2] / g.dy) ** 2)"),
    "basis_x_y_swapped": ("P = np.stack([np.ones(27), dxs[K[:, 2]], dys[K[:, 1]], dzs[K[:, 0]]], axis=1)",
                          "P = np.stack([np.ones(27), dxs[K[:, 1]], dys[K[:, 2]], dzs[K[:, 0]]], axis=1)"),
    "no_inward_shift_at_walls": ("    m = min(max(m, 1), n - 2)\n", "    m = m\n"),
    "no_periodic_image": ("        d = d - length * np.round(d / length)\n", "        d = d\n"),
    "spread_without_node_volume": ("phi * F * dv / (g.dx * g.dy * vz[kz])", "phi * F * dv / (g.dx * g.dy)"),
    "spread_with_the_middle_plane_volume": ("phi * F * dv / (g.dx * g.dy * vz[kz])",
                                            "phi * F * dv / (g.dx * g.dy * vz[kz[13]])"),
    "u_on_cell_centres": ("x = np.arange(g.nx) * g.dx + (0.0 if comp == 0 else 0.5 * g.dx)",
                          "x = np.arange(g.nx) * g.dx + 0.5 * g.dx"),
    "w_on_cell_centres": ("z = g.zc[:-1].copy() if comp == 2 else g.zm.copy()", "z = g.zm.copy()"),
    "w_face_volume_by_dz": ("    if comp != 2:\n        return g.dz.copy()", "    if True:\n        return g.dz.copy()"),
}


def _mutated_module(old, new):
    src = inspect.getsource(I)
    assert src.count(old) == 1, old
    mod = types.ModuleType("ibm_mutant")
    mod.__dict__["__package__"] = "oracle"
    exec(compile(src.replace(old, new), "ibm_mutant", "exec"), mod.__dict__)
    return mod


def test_unmutated_oracle_passes_the_subset():
    assert _run_pins() == 0


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, monkeypatch):
    mod = _mutated_module(*MUTANTS[name])
    for fn in ("node_coords", "node_volumes_z", "_window", "shape_functions", "interpolate", "spread"):
        monkeypatch.setattr(I, fn, getattr(mod, fn))
    assert _run_pins() >= 1, name
