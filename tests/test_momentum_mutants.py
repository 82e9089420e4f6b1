"""Plant plausible mistakes in the momentum right-hand-side oracle (on the
CPU, by editing a copy of its source) and check that its pins catch each."""
import inspect
import types

import numpy as np
import pytest

import oracle.momentum_oracle as M
import test_momentum_oracle as pins
from oracle import PERIODIC, WALL


def _run_pins():
    checks = [
        pins.test_x_flux_of_a_sine_closed_form,
        pins.test_z_flux_of_a_sine_closed_form,
        pins.test_cross_fluxes_are_central_differences,
        pins.test_z_interpolation_reproduces_a_linear_profile,
        lambda: pins.test_fluxes_telescope((PERIODIC, PERIODIC)),
        lambda: pins.test_energy_conservation_uniform_grid((WALL, WALL)),
        lambda: pins.test_energy_conservation_uniform_grid((PERIODIC, WALL)),
        pins.test_rhs_weights,
    ]
    failed = 0
    for c in checks:
        try:
            c()
        except (AssertionError, ValueError, IndexError):
            failed += 1
    return failed


# (original text, mutated text): each a plausible slip in the discretisation
MUTANTS = {
    "zi_weights_swapped": ("wlo = dz[1:] / (dz[:-1] + dz[1:])", "wlo = dz[:-1] / (dz[:-1] + dz[1:])"),
    "w_volume_by_dz": ("nw = (fzz - sz(fzz, -1)) / h", "nw = (fzz - sz(fzz, -1)) / dz"),
    "u_centre_wrong_neighbour": ("uc = 0.5 * (u + sx(u, 1))", "uc = 0.5 * (u + sx(u, -1))"),
    "y_flux_sign": ("nu += (sy(fxy, 1) - fxy) / g.dy", "nu += (fxy - sy(fxy, 1)) / g.dy"),
    "v_x_edge_unaveraged": ("fyx = vxe * uye", "fyx = v * uye"),
    "w_y_flux_no_interp": ("fzy = 0.5 * (sy(w, -1) + w) * _zi(v, g)", "fzy = 0.5 * (sy(w, -1) + w) * v"),
    "viscous_sign": ("r = dt * (-adv + laplacian_component(q, g, c) / re)",
                     "r = dt * (-adv - laplacian_component(q, g, c) / re)"),
}


def _mutated_module(old, new):
    src = inspect.getsource(M)
    assert src.count(old) == 1, old
    mod = types.ModuleType("momentum_mutant")
    mod.__dict__["__package__"] = "oracle"
    exec(compile(src.replace(old, new), "momentum_mutant", "exec"), mod.__dict__)
    return mod


def test_unmutated_oracle_passes_the_subset():
    assert _run_pins() == 0


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, monkeypatch):
    mod = _mutated_module(*MUTANTS[name])
    for fn in ("convective", "momentum_rhs", "laplacian_component", "_zi", "_shift"):
        monkeypatch.setattr(M, fn, getattr(mod, fn))
    assert _run_pins() >= 1, name
