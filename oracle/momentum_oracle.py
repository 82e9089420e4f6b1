"""Plain FP64 CPU oracle for the explicit part of the momentum step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  The HIP library
never imports it and shares no code, table or constant generator with it.

What is computed (paper, Sec. 2.1, eq. NSdiscr0): the convective term is
advanced explicitly by a two-level Adams-Bashforth scheme with weights
gamma = 3/2, rho = -1/2, and the viscous term by Crank-Nicolson.  With the
pressure left to the projection (fractional step, Sec. 2.1), the provisional
increment du = u* - u^n solves

    (I - beta Lap) du = dt [ -(gamma N^n + rho N^{n-1}) + (1/Re) Lap u^n ],
    beta = dt / (2 Re),   N = div(u u),

and this module computes the right-hand side (and N^n, kept for the next
step).  The left-hand side is the implicit viscous step (viscous_oracle).

Readings taken here (the paper names central second-order differences on a
staggered mesh, Sec. 2.1, and is silent on the rest):
  * N in divergence (conservative) form on each component's control volume:
    u-volume around x-face i spans cell centres i-1, i; fluxes of u-momentum
    through its faces are products of two-point averages: (u u) at cell
    centres from the mean of the two adjacent faces, (u v) at the xy edges from
    the y-mean of u and the x-mean of v, (u w) at the xz edges from the
    z-interpolated u and the x-mean of w; likewise for v and w;
  * z interpolation of a centre value to a z face: linear in z,
    q_f = (dz_k q_{k-1} + dz_{k-1} q_k) / (dz_{k-1} + dz_k); the z divergence of
    the u and v volumes divides by dz_k, of the w volume by h_k;
  * walls carry no flux of any momentum (zero normal velocity on the wall);
  * Lap = L_x + L_y + L_z with the component's operators of the viscous step;
  * dead wall faces: right-hand side and N are 0 there.
"""
from __future__ import annotations

import numpy as np

from .fsei_oracle import WALL, Grid
from .viscous_oracle import AXIS_OF, dead_mask, second_difference


def _shift(a, off, axis, periodic):
    """b[..., i, ...] = a[..., i + off, ...]; outside the grid 0 (wall) or
    wrapped (periodic)."""
    b = np.roll(a, -off, axis=axis)
    if not periodic:
        n = a.shape[axis]
        idx = [slice(None)] * 3
        if off > 0:
            idx[axis] = slice(n - off, n)
        else:
            idx[axis] = slice(0, -off)
        b[tuple(idx)] = 0.0
    return b


def _zi(q, g: Grid):
    """Centre values q_k linearly interpolated to z faces k (k = 1..nz-1);
    face 0 gets 0 (wall; it is always multiplied by w = 0 there)."""
    out = np.zeros_like(q)
    dz = g.dz
    wlo = dz[1:] / (dz[:-1] + dz[1:])      # weight of q_{k-1} at face k
    whi = dz[:-1] / (dz[:-1] + dz[1:])     # weight of q_k
    out[1:] = wlo[:, None, None] * q[:-1] + whi[:, None, None] * q[1:]
    return out


def convective(u, v, w, g: Grid):
    """(N_u, N_v, N_w) = div of the momentum fluxes on each component's
    control volume; dead wall faces 0."""
    px, py = g.bcx != WALL, g.bcy != WALL
    mu, mv, mw = (dead_mask(g, c) for c in range(3))
    u = np.where(mu, 0.0, u)
    v = np.where(mv, 0.0, v)
    w = np.where(mw, 0.0, w)
    dz = g.dz[:, None, None]
    h = g.h.copy()
    h[0] = 1.0
    h = h[:, None, None]
    sx = lambda a, o: _shift(a, o, 2, px)
    sy = lambda a, o: _shift(a, o, 1, py)
    sz = lambda a, o: _shift(a, o, 0, False)

    # ---- u at x-face i (cell centres i-1 and i around it)
    uc = 0.5 * (u + sx(u, 1))                         # u at centre i (faces i, i+1)
    fxx = uc * uc                                     # flux through centre i
    nu = (fxx - sx(fxx, -1)) / g.dx                   # centre i minus centre i-1
    # y: edge (i, j) between y-cells j-1 and j: u averaged in y, v averaged in x
    uy = 0.5 * (sy(u, -1) + u)
    vx = 0.5 * (sx(v, -1) + v)
    fxy = uy * vx                                     # at y-face j of the u-volume
    nu += (sy(fxy, 1) - fxy) / g.dy
    # z: edge (i, k) at z-face k: u interpolated in z, w averaged in x
    fxz = _zi(u, g) * 0.5 * (sx(w, -1) + w)
    nu += (sz(fxz, 1) - fxz) / dz

    # ---- v at y-face j
    vc = 0.5 * (v + sy(v, 1))
    fyy = vc * vc
    nv = (fyy - sy(fyy, -1)) / g.dy
    vxe = 0.5 * (sx(v, -1) + v)                       # v averaged in x to x-face i
    uye = 0.5 * (sy(u, -1) + u)                       # u averaged in y to y-face j
    fyx = vxe * uye                                   # at x-face i of the v-volume
    nv += (sx(fyx, 1) - fyx) / g.dx
    fyz = _zi(v, g) * 0.5 * (sy(w, -1) + w)
    nv += (sz(fyz, 1) - fyz) / dz

    # ---- w at z-face k (cell centres k-1 and k around it)
    wc = 0.5 * (w + sz(w, 1))                         # w at centre k
    fzz = wc * wc
    nw = (fzz - sz(fzz, -1)) / h
    fzx = 0.5 * (sx(w, -1) + w) * _zi(u, g)           # at x-face i, z-face k
    nw += (sx(fzx, 1) - fzx) / g.dx
    fzy = 0.5 * (sy(w, -1) + w) * _zi(v, g)
    nw += (sy(fzy, 1) - fzy) / g.dy

    return (np.where(mu, 0.0, nu), np.where(mv, 0.0, nv), np.where(mw, 0.0, nw))


def laplacian_component(q, g: Grid, comp: int):
    """(L_x + L_y + L_z) q with the component's viscous-step operators."""
    q = np.where(dead_mask(g, comp), 0.0, q)
    out = np.zeros_like(q)
    for d in ("x", "y", "z"):
        L = second_difference(g, comp, d)
        b = np.moveaxis(q, AXIS_OF[d], -1)
        out += np.moveaxis(b @ L.T, -1, AXIS_OF[d])
    return np.where(dead_mask(g, comp), 0.0, out)


def momentum_rhs(u, v, w, nprev, g: Grid, dt: float, re: float, gamma: float = 1.5, rho: float = -0.5):
    """dt [ -(gamma N^n + rho N^{n-1}) + (1/Re) Lap u^n ] per component, and
    N^n.  nprev: (N_u, N_v, N_w) of the previous step (ignored when rho = 0)."""
    n = convective(u, v, w, g)
    out = []
    for c, q in enumerate((u, v, w)):
        adv = gamma * n[c] + (rho * nprev[c] if rho != 0.0 else 0.0)
        r = dt * (-adv + laplacian_component(q, g, c) / re)
        out.append(np.where(dead_mask(g, c), 0.0, r))
    return tuple(out), n
