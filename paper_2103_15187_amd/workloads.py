"""Seeded synthetic inputs for the pressure projection.

This module holds only input recipes (grids, random fields); none of the
projection's arithmetic.  Tests, the benchmark and the CPU reference all draw
their inputs from here, so both sides of every comparison see the same arrays.

Grids are shaped like the paper's heart domain (Sec. 5: periodic x,y and walls
in z for its own runs; Sec. 5 gives a 96 x 96 x 156 mm^3 box, i.e. an aspect
ratio of 4 : 4 : 6.5 in units of the 24 mm mitral diameter).  The paper states
no wall-normal stretching law; a two-sided tanh clustering is used:

    zc_k = (Lz/2) [1 + tanh(s (2k/nz - 1)) / tanh(s)],  k = 0..nz.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

PERIODIC = 0
WALL = 1


def tanh_faces(nz: int, lz: float, s: float) -> np.ndarray:
    """nz+1 strictly increasing z-face coordinates clustered toward both walls."""
    k = np.arange(nz + 1, dtype=np.float64)
    if s == 0.0:
        return lz * k / nz
    return 0.5 * lz * (1.0 + np.tanh(s * (2.0 * k / nz - 1.0)) / np.tanh(s))


@dataclass(frozen=True)
class GridSpec:
    nx: int
    ny: int
    nz: int
    bcx: int
    bcy: int
    lx: float
    ly: float
    lz: float
    stretch: float

    @property
    def dx(self) -> float:
        return self.lx / self.nx

    @property
    def dy(self) -> float:
        return self.ly / self.ny

    def zc(self) -> np.ndarray:
        return tanh_faces(self.nz, self.lz, self.stretch)

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)


# The five workloads.  Sizes count pressure cells (nx*ny*nz).
CONFIGS = {
    # 64^3 box of unit size, walls everywhere, z tanh factor 1.5
    "C1": GridSpec(64, 64, 64, WALL, WALL, 1.0, 1.0, 1.0, 1.5),
    # 256 x 256 x 384, x periodic, y and z walls, tanh 2.0
    "C2": GridSpec(256, 256, 384, PERIODIC, WALL, 4.0, 4.0, 6.5, 2.0),
    # 512 x 512 x 768, walls everywhere, tanh 2.5 (headline workload)
    "C3": GridSpec(512, 512, 768, WALL, WALL, 4.0, 4.0, 6.5, 2.5),
    # adjoint workloads: x periodic, y wall, z wall, tanh 2.0
    "C4a": GridSpec(128, 128, 192, PERIODIC, WALL, 4.0, 4.0, 6.5, 2.0),
    "C4b": GridSpec(256, 256, 384, PERIODIC, WALL, 4.0, 4.0, 6.5, 2.0),
    # 768 x 768 x 1024, walls everywhere, tanh 3.0
    "C5": GridSpec(768, 768, 1024, WALL, WALL, 4.0, 4.0, 6.5, 3.0),
}
SEEDS = {"C1": 1, "C2": 2, "C3": 3, "C4a": 4, "C4b": 4, "C5": 5}


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def dead_face_masks(spec: GridSpec):
    """Masks of the stored face entries that lie on walls (x walls: u[:,:,0];
    y walls: v[:,0,:]; z walls: w[0,:,:])."""
    mu = np.zeros(spec.shape, dtype=bool)
    mv = np.zeros(spec.shape, dtype=bool)
    mw = np.zeros(spec.shape, dtype=bool)
    if spec.bcx == WALL:
        mu[:, :, 0] = True
    if spec.bcy == WALL:
        mv[:, 0, :] = True
    mw[0, :, :] = True
    return mu, mv, mw


def random_velocity(spec: GridSpec, seed: int, dtype=np.float64):
    """u*, v*, w* ~ N(0,1) i.i.d. on every stored face, wall faces set to 0."""
    g = rng(seed)
    u = g.standard_normal(spec.shape, dtype=np.float64)
    v = g.standard_normal(spec.shape, dtype=np.float64)
    w = g.standard_normal(spec.shape, dtype=np.float64)
    for a, m in zip((u, v, w), dead_face_masks(spec)):
        a[m] = 0.0
    return u.astype(dtype, copy=False), v.astype(dtype, copy=False), w.astype(dtype, copy=False)


def add_jet(spec: GridSpec, w: np.ndarray, amplitude=10.0, width_frac=0.05):
    """Localised Gaussian jet on the w faces (valve-inflow stand-in):
    w += A exp(-|x - x0|^2 / (2 sigma^2)), sigma = width_frac * Lx,
    x0 = (Lx/2, Ly/2, Lz/3), evaluated at the w-face positions."""
    sigma = width_frac * spec.lx
    x = (np.arange(spec.nx) + 0.5) * spec.dx
    y = (np.arange(spec.ny) + 0.5) * spec.dy
    z = spec.zc()[:-1]
    gx = np.exp(-((x - spec.lx / 2) ** 2) / (2 * sigma ** 2))
    gy = np.exp(-((y - spec.ly / 2) ** 2) / (2 * sigma ** 2))
    gz = np.exp(-((z - spec.lz / 3) ** 2) / (2 * sigma ** 2))
    jet = amplitude * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    jet[0] = 0.0
    w += jet.astype(w.dtype)
    return w


def c3_velocity(spec: GridSpec = CONFIGS["C3"], seed: int = SEEDS["C3"]):
    u, v, w = random_velocity(spec, seed)
    add_jet(spec, w)
    return u, v, w


def _cell_positions(spec: GridSpec):
    x = (np.arange(spec.nx) + 0.5) * spec.dx
    y = (np.arange(spec.ny) + 0.5) * spec.dy
    zc = spec.zc()
    z = 0.5 * (zc[1:] + zc[:-1])
    return x, y, z


def remove_volume_mean(spec: GridSpec, f: np.ndarray) -> np.ndarray:
    """Subtract the cell-volume-weighted average (input preparation only)."""
    dz = np.diff(spec.zc())
    plane_sums = f.sum(axis=(1, 2))
    mean = float((dz * plane_sums).sum() / (dz.sum() * spec.nx * spec.ny))
    return f - mean


def rhs_modes(spec: GridSpec, seed: int, nmodes=32, kmax=8, noise=1e-3):
    """Sum of `nmodes` seeded low-wavenumber modes plus N(0, noise^2):
    A_q cos(2 pi m x/Lx + phi) cos(pi n y/Ly) cos(pi l z/Lz), m,n,l ~ U{0..kmax-1},
    A ~ N(0,1), phi ~ U(0, 2 pi); volume-weighted mean removed."""
    g = rng(seed)
    x, y, z = _cell_positions(spec)
    f = np.zeros(spec.shape)
    xfun = (lambda m, ph: np.cos(2 * np.pi * m * x / spec.lx + ph)) if spec.bcx == PERIODIC \
        else (lambda m, ph: np.cos(np.pi * m * x / spec.lx))
    yfun = (lambda n, ph: np.cos(2 * np.pi * n * y / spec.ly + ph)) if spec.bcy == PERIODIC \
        else (lambda n, ph: np.cos(np.pi * n * y / spec.ly))
    for _ in range(nmodes):
        m, n, l = g.integers(0, kmax, size=3)
        a = g.standard_normal()
        ph = g.uniform(0, 2 * np.pi)
        f += a * (np.cos(np.pi * l * z / spec.lz)[:, None, None]
                  * yfun(n, 0.0)[None, :, None] * xfun(m, ph)[None, None, :])
    f += noise * g.standard_normal(spec.shape)
    return remove_volume_mean(spec, f)


def rhs_powerlaw(spec: GridSpec, seed: int, nmodes=64):
    """Multi-scale field: sum over m,n,l < nmodes (not all zero) of
    N(0,1) |k|^{-11/6} cos(pi m x/Lx) cos(pi n y/Ly) cos(pi l z/Lz), so the
    shell spectrum falls as k^{-5/3}; synthesised separably; mean removed."""
    g = rng(seed)
    x, y, z = _cell_positions(spec)
    m = np.arange(nmodes)
    kx = np.pi * m / spec.lx
    ky = np.pi * m / spec.ly
    kz = np.pi * m / spec.lz
    kk = np.sqrt(kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2)
    kk[0, 0, 0] = 1.0
    amp = g.standard_normal((nmodes, nmodes, nmodes)) * kk ** (-11.0 / 6.0)
    amp[0, 0, 0] = 0.0
    cx = np.cos(np.outer(m, np.pi * x / spec.lx))     # (nmodes, nx)
    cy = np.cos(np.outer(m, np.pi * y / spec.ly))
    cz = np.cos(np.outer(m, np.pi * z / spec.lz))
    # f[k,j,i] = sum_{l,n,m} amp[l,n,m] cz[l,k] cy[n,j] cx[m,i]
    t = np.tensordot(amp, cx, axes=([2], [0]))          # (l, n, nx)
    t = np.tensordot(t, cy, axes=([1], [0]))            # (l, nx, ny)
    f = np.tensordot(cz, t, axes=([0], [0]))            # (nz, nx, ny)
    f = np.ascontiguousarray(np.swapaxes(f, 1, 2))
    return remove_volume_mean(spec, f)


def face_weights_random(spec: GridSpec, seed: int):
    """Positive loss weights omega ~ U(0.5, 1.5) per face (adjoint workload)."""
    g = rng(seed + 1000)
    return tuple(g.uniform(0.5, 1.5, size=spec.shape) for _ in range(3))


def small_spec(nx, ny, nz, bcx=WALL, bcy=WALL, lx=None, ly=None, lz=1.0, stretch=1.5):
    """Helper for tiny test grids."""
    return GridSpec(nx, ny, nz, bcx, bcy, lx if lx else 1.0, ly if ly else 1.0, lz, stretch)


def uniform_markers(spec: GridSpec, nb: int, seed: int) -> np.ndarray:
    """nb Lagrangian marker positions (nb, 3), uniform in the domain."""
    g = rng(seed)
    zc = spec.zc()
    return np.stack([g.uniform(0, spec.lx, nb), g.uniform(0, spec.ly, nb), g.uniform(zc[0], zc[-1], nb)], 1)


def spheroid_markers(spec: GridSpec, radius: float = 1.2, height: float = 2.4):
    """Markers of a wet surface: the centroids of a triangulated prolate
    spheroid (semi-axes radius, radius, height) centred in the domain, with
    about one triangle per dx * dy of surface, since the paper refines its
    surface meshes until every tile is smaller than the local grid spacing
    (Sec. 4).  A latitude-longitude mesh: each quad is split in two triangles;
    markers come out in mesh order (neighbours in memory are neighbours on the
    surface; the collapsed triangles at the poles are dropped), and each marker's volume is its triangle's area times dx.

    Returns (xb (nb, 3), dv (nb,))."""
    c0 = np.array([0.5 * spec.lx, 0.5 * spec.ly, 0.5 * spec.zc()[-1]])
    h = np.sqrt(spec.dx * spec.dy)
    # meridian length (Ramanujan's perimeter of the ellipse, halved) and equator
    a, b = radius, height
    meridian = 0.5 * np.pi * (3 * (a + b) - np.sqrt((3 * a + b) * (a + 3 * b)))
    nt = max(2, int(np.ceil(meridian / (1.2 * h))))
    npz = max(3, int(np.ceil(2 * np.pi * a / (1.2 * h))))
    th = np.linspace(0.0, np.pi, nt + 1)
    ph = np.linspace(0.0, 2 * np.pi, npz + 1)
    T, P = np.meshgrid(th, ph, indexing="ij")
    V = np.stack([a * np.sin(T) * np.cos(P), a * np.sin(T) * np.sin(P), b * np.cos(T)], -1) + c0
    p00, p01, p10, p11 = V[:-1, :-1], V[:-1, 1:], V[1:, :-1], V[1:, 1:]
    tri = np.stack([np.stack([p00, p10, p11], -2), np.stack([p00, p11, p01], -2)], 2)   # (nt, np, 2, 3, 3)
    tri = tri.reshape(-1, 3, 3)
    area = 0.5 * np.linalg.norm(np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0]), axis=1)
    keep = area > 1e-12 * h * h          # the collapsed triangles at the two poles
    xb = tri[keep].mean(axis=1)
    return np.ascontiguousarray(xb), area[keep] * spec.dx
