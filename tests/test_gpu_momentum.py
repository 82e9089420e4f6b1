"""Parity of the explicit momentum right-hand side (fsei_momentum_rhs, through
the C ABI) with the FP64 oracle, and of one whole fractional step built from
the library's calls (right-hand side, implicit viscous step, projection).

Bar: <= 1e-12 of max |oracle| element by element (a few tens of FP64
operations per value).  At 512 x 512 x 768 sampled z-planes are compared with
the oracle evaluated on a slab of planes around each (the stencil reaches one
plane up and down), including both walls."""
import numpy as np
import pytest

import oracle
from oracle import PERIODIC, WALL
from oracle import momentum as MO
from oracle import viscous as V
from paper_2103_15187_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BCS = [(WALL, WALL), (PERIODIC, WALL), (WALL, PERIODIC), (PERIODIC, PERIODIC)]
DIMS = [(8, 6, 5), (24, 18, 20), (27, 9, 33), (2, 3, 4), (64, 48, 40), (256, 32, 9), (128, 48, 7)]


def fsei():
    from paper_2103_15187_amd import fsei as F
    return F


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=torch.float64)


def host(t):
    return t.detach().cpu().numpy()


def check(got, ref, what):
    scale = max(np.abs(ref).max(), 1e-300)
    err = np.abs(got - ref).max()
    assert err <= 1e-12 * scale, (what, err / scale)


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("dims", DIMS)
def test_momentum_rhs_matches_oracle(dims, bc):
    nx, ny, nz = dims
    spec = W.GridSpec(nx, ny, nz, bc[0], bc[1], 1.3, 0.9, 1.7, 2.2)
    g = oracle.Grid(nx, ny, nz, bc[0], bc[1], spec.dx, spec.dy, spec.zc())
    F = fsei()
    plan = F.Plan.from_spec(spec)
    rng = W.rng(21 + nx + ny + nz)
    u, v, w = (rng.standard_normal(spec.shape) for _ in range(3))   # dead faces hold garbage
    prev = tuple(rng.standard_normal(spec.shape) for _ in range(3))
    for gamma, rho in ((1.5, -0.5), (1.0, 0.0)):
        print(f"momentum dims={dims} bc={bc} gamma={gamma}", flush=True)
        n = [dev(a) for a in prev]
        r = [torch.empty_like(n[0]) for _ in range(3)]
        plan.momentum_rhs(dev(u), dev(v), dev(w), n, r, dt=0.013, re=70.0, gamma=gamma, rho=rho)
        torch.cuda.synchronize()
        (rr, nn) = MO.momentum_rhs(u, v, w, prev, g, dt=0.013, re=70.0, gamma=gamma, rho=rho)
        for c in range(3):
            check(host(r[c]), rr[c], ("rhs", c))
            check(host(n[c]), nn[c], ("N", c))


def test_fractional_step_composition():
    """u^n -> rhs -> (I - bLx)(I - bLy)(I - bLz) du = rhs -> u* = u^n + du ->
    projection, every step in the library's kernels, against the same chain in
    the oracle."""
    spec = W.GridSpec(24, 18, 20, PERIODIC, WALL, 2.0, 1.5, 1.7, 2.0)
    g = oracle.Grid(spec.nx, spec.ny, spec.nz, spec.bcx, spec.bcy, spec.dx, spec.dy, spec.zc())
    F = fsei()
    plan = F.Plan.from_spec(spec)
    rng = W.rng(99)
    u, v, w = (rng.standard_normal(spec.shape) for _ in range(3))
    u, v, w, _ = oracle.project(u, v, w, g)
    prev = tuple(rng.standard_normal(spec.shape) for _ in range(3))
    dt, re = 0.01, 100.0
    beta = dt / (2 * re)
    # oracle chain
    (rr, _) = MO.momentum_rhs(u, v, w, prev, g, dt, re)
    star = [q + V.viscous_solve(rr[c], g, c, beta) for c, q in enumerate((u, v, w))]
    ou, ov, ow, op = oracle.project(*star, g, dt=dt)
    # library chain: rhs, implicit solve added to u^n in its last pass (u*), projection
    ud = [dev(a) for a in (u, v, w)]
    n = [dev(a) for a in prev]
    r = [torch.empty_like(ud[0]) for _ in range(3)]
    plan.momentum_rhs(*ud, n, r, dt=dt, re=re)
    star_d = [a.clone() for a in ud]
    for c in range(3):
        plan.viscous_solve_add(r[c], star_d[c], c, beta)
    ud = star_d
    p = plan.project(*ud, dt=dt)
    torch.cuda.synchronize()
    for got, ref in zip(ud + [p], (ou, ov, ow, op)):
        check(host(got), ref, "step")


@pytest.mark.timeout(400)
def test_c3_momentum_rhs_sampled_planes():
    spec = W.CONFIGS["C3"]
    zc = spec.zc()
    F = fsei()
    plan = F.Plan.from_spec(spec)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    ud = [torch.randn(spec.shape, dtype=torch.float64, device="cuda", generator=gen) for _ in range(3)]
    pd = [torch.randn(spec.shape, dtype=torch.float64, device="cuda", generator=gen) for _ in range(3)]
    n = [a.clone() for a in pd]
    r = [torch.empty_like(ud[0]) for _ in range(3)]
    plan.momentum_rhs(*ud, n, r, dt=1e-3, re=300.0)
    torch.cuda.synchronize()
    for k in (0, 1, 2, 383, spec.nz - 2, spec.nz - 1):
        lo, hi = max(0, k - 2), min(spec.nz, k + 3)
        print(f"C3 momentum plane {k}", flush=True)
        gs = oracle.Grid(spec.nx, spec.ny, hi - lo, spec.bcx, spec.bcy, spec.dx, spec.dy, zc[lo:hi + 1])
        sl = lambda t: host(t[lo:hi])
        (rr, nn) = MO.momentum_rhs(*(sl(a) for a in ud), tuple(sl(a) for a in pd), gs, dt=1e-3, re=300.0)
        for c in range(3):
            if c == 2 and k == 0:
                assert torch.all(r[2][0] == 0) and torch.all(n[2][0] == 0)
                continue
            check(host(r[c][k]), rr[c][k - lo], ("rhs", c, k))
            check(host(n[c][k]), nn[c][k - lo], ("N", c, k))
