"""Plain FP64 CPU oracle for the immersed-boundary moving-least-squares
(IB-MLS) transfer between Lagrangian markers and the staggered Eulerian grid.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  The HIP library
never imports it and shares no code, table or constant generator with it.

What is computed (paper, Sec. 2.1, eq. interpv and Fig. mls): around each
marker x_b a support of n x n x n = 27 Eulerian nodes of the velocity
component's own (staggered) lattice; the velocity at the marker is
sum_k phi_k(x_b) u(x_k), with MLS transfer operators built on the linear basis
p = [1, x, y, z] and an exponential weight centred on the marker.  The IB force
computed at the marker is transferred back to the same nodes as a distributed
forcing (Sec. 2.1).

The MLS operator, written out (basis shifted to the marker, p(x_b) = e_0):
    A     = sum_k W_k p_k p_k^T,        p_k = [1, x_k - x_b, y_k - y_b, z_k - z_b]
    phi_k = e_0^T A^-1 p_k W_k.

Readings taken here (the paper defers the MLS details to a citation):
  * support: along each axis the 3 consecutive nodes whose middle one is the
    node nearest the marker, shifted inwards at walls (always 3 in-domain
    nodes) and wrapped in periodic directions (displacements to the nearest
    periodic image);
  * node positions of component c: its own axis on faces (x_i = i dx, z faces
    zc[k]), the other axes on cell centres ((i + 1/2) dx, zm[k]);
  * weight W_k = exp(-(dx_k / dx)^2 - (dy_k / dy)^2 - (dz_k / hz)^2), with dx_k the
    marker-node displacement and hz the z spacing of the support's middle
    node (cell width dz for centres, centre distance h for faces);
  * spreading: f_k += phi_k F_b dV_b / V_k, with V_k the control volume of
    node k (dx dy dz_k for u, v; dx dy h_k for w, h_0 = dz_0 / 2); this makes
    spreading the volume-weighted transpose of interpolation.
"""
from __future__ import annotations

import numpy as np

from .fsei_oracle import WALL, Grid


def node_coords(g: Grid, comp: int):
    """1-D node coordinates (x, y, z) of component comp's lattice."""
    x = np.arange(g.nx) * g.dx + (0.0 if comp == 0 else 0.5 * g.dx)
    y = np.arange(g.ny) * g.dy + (0.0 if comp == 1 else 0.5 * g.dy)
    z = g.zc[:-1].copy() if comp == 2 else g.zm.copy()
    return x, y, z


def node_volumes_z(g: Grid, comp: int):
    """z extent of the control volume of each node (dz for centres, h for
    faces with h_0 = dz_0 / 2)."""
    if comp != 2:
        return g.dz.copy()
    h = g.h.copy()
    h[0] = 0.5 * g.dz[0]
    return h


def _window(coords, xb, n, periodic, length):
    """Indices (3,) of the support along one axis and the displacements
    x_node - x_b (nearest periodic image)."""
    if periodic:
        d = coords - xb
        d = d - length * np.round(d / length)
        m = int(np.argmin(np.abs(d)))
        idx = np.array([(m - 1) % n, m, (m + 1) % n])
        return idx, d[idx]
    m = int(np.argmin(np.abs(coords - xb)))
    m = min(max(m, 1), n - 2)
    idx = np.array([m - 1, m, m + 1])
    return idx, coords[idx] - xb


def shape_functions(g: Grid, comp: int, xb):
    """For one marker: flat indices (27,) into the (nz, ny, nx) field and the
    MLS transfer operators phi (27,)."""
    x, y, z = node_coords(g, comp)
    ix, dxs = _window(x, xb[0], g.nx, g.bcx != WALL, g.nx * g.dx)
    iy, dys = _window(y, xb[1], g.ny, g.bcy != WALL, g.ny * g.dy)
    iz, dzs = _window(z, xb[2], g.nz, False, None)
    hz = node_volumes_z(g, comp)[iz[1]]
    K = np.array([(kk, jj, ii) for kk in range(3) for jj in range(3) for ii in range(3)])
    P = np.stack([np.ones(27), dxs[K[:, 2]], dys[K[:, 1]], dzs[K[:, 0]]], axis=1)
    Wk = np.exp(-(P[:, 1] / g.dx) ** 2 - (P[:, 2] / g.dy) ** 2 - (P[:, 3] / hz) ** 2)
    A = (P * Wk[:, None]).T @ P
    e0 = np.array([1.0, 0.0, 0.0, 0.0])
    phi = (np.linalg.solve(A, e0) @ P.T) * Wk            # A symmetric: e0^T A^-1 p_k W_k
    flat = (iz[K[:, 0]] * g.ny + iy[K[:, 1]]) * g.nx + ix[K[:, 2]]
    return flat, phi


def interpolate(field, g: Grid, comp: int, xb):
    """u(x_b) = sum_k phi_k u(x_k) for every marker (xb: (nb, 3))."""
    f = np.asarray(field, dtype=np.float64).reshape(-1)
    out = np.empty(len(xb))
    for b, x in enumerate(np.asarray(xb, dtype=np.float64)):
        flat, phi = shape_functions(g, comp, x)
        out[b] = phi @ f[flat]
    return out


def spread(g: Grid, comp: int, xb, fb, dvb):
    """Distributed forcing: f_k = sum_b phi_k(x_b) F_b dV_b / V_k."""
    out = np.zeros(g.nx * g.ny * g.nz)
    vz = node_volumes_z(g, comp)
    for x, F, dv in zip(np.asarray(xb, dtype=np.float64), fb, dvb):
        flat, phi = shape_functions(g, comp, x)
        kz = flat // (g.nx * g.ny)
        np.add.at(out, flat, phi * F * dv / (g.dx * g.dy * vz[kz]))
    return out.reshape(g.shape)
