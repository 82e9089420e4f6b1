"""Plain FP64 CPU oracle for the implicit viscous step (approximate factorisation).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  The HIP library
never imports it and shares no code, table or constant generator with it.

What is computed (paper, Sec. 2.1, eq. NSdiscr0, and Sec. 3 on the solver's
parallelisation): the viscous term is advanced by Crank-Nicolson, which makes
the momentum update a Helmholtz-type problem (I - beta Lap) du = rhs with
beta = dt / (2 Re).  The paper avoids the 3-D sparse solve by an approximate
factorisation into one tridiagonal operator per direction,

    (I - beta L_x)(I - beta L_y)(I - beta L_z) du = rhs,

inverted direction by direction with Thomas' algorithm, with a
Sherman-Morrison correction in the periodic directions.  This oracle builds
each 1-D operator as a dense FP64 matrix from the staggered second-difference
stencil and applies its inverse line by line with numpy.linalg.solve (the
plain definition; no Thomas, no Sherman-Morrison, no factorisation reuse).

Readings taken here (the paper is silent on them):
  * component c in {0: u, 1: v, 2: w} sits on the low face of its cell along
    its own axis and at cell centres along the other two (same layout as the
    projection oracle, arrays (nz, ny, nx));
  * along its own axis: face values, Dirichlet zero at walls (the stored wall
    face is dead: ignored on input, 0 on output; the opposite wall face is not
    stored and is 0);  z faces: (d2w)_k = ((w_{k+1}-w_k)/dz_k -
    (w_k-w_{k-1})/dz_{k-1}) / h_k;
  * along the other axes: centre values, no-slip walls through a mirrored
    ghost (q_ghost = -q at the wall-adjacent centre, i.e. a wall flux
    2 q / dz over the half cell);  z centres: (d2q)_k = ((q_{k+1}-q_k)/h_{k+1}
    - (q_k-q_{k-1})/h_k) / dz_k;
  * periodic x / y: cyclic three-point stencil; z is always walled;
  * beta > 0 is passed in (dt / (2 Re) for the Crank-Nicolson half).
"""
from __future__ import annotations

import numpy as np

from .fsei_oracle import WALL, Grid

AXIS_OF = {"x": 2, "y": 1, "z": 0}


def second_difference(g: Grid, comp: int, direction: str) -> np.ndarray:
    """Dense 1-D second-difference matrix L_d for component `comp` along
    `direction` (n x n), with the rows of a dead wall face set to zero."""
    own = {"x": 0, "y": 1, "z": 2}[direction] == comp
    if direction in ("x", "y"):
        n = g.nx if direction == "x" else g.ny
        d = g.dx if direction == "x" else g.dy
        bc = g.bcx if direction == "x" else g.bcy
        L = np.zeros((n, n))
        for i in range(n):
            for off in (-1, 1):
                j = i + off
                if 0 <= j < n:
                    L[i, j] += 1.0 / d**2
                    L[i, i] -= 1.0 / d**2
                elif bc != WALL:                      # periodic wrap
                    L[i, j % n] += 1.0 / d**2
                    L[i, i] -= 1.0 / d**2
                elif own:                             # neighbour is a wall face: value 0
                    L[i, i] -= 1.0 / d**2
                else:                                 # mirrored ghost: -q_i
                    L[i, i] -= 2.0 / d**2
        if own and bc == WALL:
            L[0, :] = 0.0                             # face 0 is the wall: dead
            L[:, 0] = 0.0
        return L
    # z: stretched, walls at both ends
    n = g.nz
    L = np.zeros((n, n))
    if own:
        # w on faces k (face k at zc[k]); w_0 = w_nz = 0
        for k in range(1, n):
            lo = 1.0 / (g.dz[k - 1] * g.h[k])         # coefficient of w_{k-1}
            hi = 1.0 / (g.dz[k] * g.h[k])             # coefficient of w_{k+1}
            if k - 1 >= 1:
                L[k, k - 1] = lo
            if k + 1 < n:
                L[k, k + 1] = hi
            L[k, k] = -(lo + hi)
        return L
    for k in range(n):
        if k >= 1:
            lo = 1.0 / (g.h[k] * g.dz[k])
            L[k, k - 1] = lo
        else:
            lo = 2.0 / (g.dz[0] * g.dz[0])            # wall flux over the half cell
        if k + 1 < n:
            hi = 1.0 / (g.h[k + 1] * g.dz[k])
            L[k, k + 1] = hi
        else:
            hi = 2.0 / (g.dz[k] * g.dz[k])
        L[k, k] = -(lo + hi)
    return L


def helmholtz_factor(g: Grid, comp: int, direction: str, beta: float) -> np.ndarray:
    """I - beta L_d, with a dead wall-face row made the identity (its value
    is forced to 0 through a zero right-hand side)."""
    L = second_difference(g, comp, direction)
    return np.eye(L.shape[0]) - beta * L


def dead_mask(g: Grid, comp: int) -> np.ndarray:
    """True on the dead wall faces of component `comp`."""
    m = np.zeros(g.shape, dtype=bool)
    if comp == 0 and g.bcx == WALL:
        m[:, :, 0] = True
    if comp == 1 and g.bcy == WALL:
        m[:, 0, :] = True
    if comp == 2:
        m[0, :, :] = True
    return m


def _solve_lines(M, a, axis):
    """Apply M^{-1} to every line of `a` along `axis` (numpy.linalg.solve)."""
    b = np.moveaxis(a, axis, -1)
    x = np.linalg.solve(M, b.reshape(-1, b.shape[-1]).T).T.reshape(b.shape)
    return np.moveaxis(x, -1, axis)


def _apply_lines(M, a, axis):
    b = np.moveaxis(a, axis, -1)
    return np.moveaxis(b @ M.T, -1, axis)


def viscous_solve(rhs, g: Grid, comp: int, beta: float):
    """du with (I - beta L_x)(I - beta L_y)(I - beta L_z) du = rhs on the live
    entries of component `comp`; dead wall faces are ignored and returned 0.
    The x factor is inverted first, then y, then z (eq. NSdiscr0 with the
    approximate factorisation of Sec. 3)."""
    a = np.where(dead_mask(g, comp), 0.0, np.asarray(rhs, dtype=np.float64))
    for d in ("x", "y", "z"):
        a = _solve_lines(helmholtz_factor(g, comp, d, beta), a, AXIS_OF[d])
        a = np.where(dead_mask(g, comp), 0.0, a)
    return a


def viscous_apply(q, g: Grid, comp: int, beta: float):
    """(I - beta L_x)(I - beta L_y)(I - beta L_z) q on the live entries."""
    a = np.where(dead_mask(g, comp), 0.0, np.asarray(q, dtype=np.float64))
    for d in ("z", "y", "x"):
        a = _apply_lines(helmholtz_factor(g, comp, d, beta), a, AXIS_OF[d])
        a = np.where(dead_mask(g, comp), 0.0, a)
    return a
