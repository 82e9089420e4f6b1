"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: FP64 path <= 1e-12 relative L2 against the oracle (u, v, w and p, both
with the V-mean-zero pinning); FP32+refinement <= 1e-10 relative residual;
plain FP32 <= 2e-5 relative L2 (rounding of ~40 FP32 operations per value
along the transform chain, amplified by the condition of the lowest modes
that stay in FP32)."""
import numpy as np
import pytest

import oracle
from oracle import PERIODIC, WALL
from paper_2103_15187_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BCS = [(WALL, WALL), (PERIODIC, WALL), (WALL, PERIODIC), (PERIODIC, PERIODIC)]


def fsei():
    from paper_2103_15187_amd import fsei as F
    return F


def grid_of(spec):
    return oracle.Grid(spec.nx, spec.ny, spec.nz, spec.bcx, spec.bcy, spec.dx, spec.dy, spec.zc())


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def run_project(spec, u, v, w, dt=1.0, **kw):
    F = fsei()
    plan = F.Plan.from_spec(spec, **kw)
    dtype = torch.float32 if kw.get("precision") == F.PREC_FP32 else torch.float64
    ud, vd, wd = dev(u, dtype), dev(v, dtype), dev(w, dtype)
    out = plan.project(ud, vd, wd, dt=dt, info=True)
    torch.cuda.synchronize()
    p, info = out
    return host(ud), host(vd), host(wd), host(p), info


SMALL = [(4, 6, 8), (8, 8, 8), (6, 3, 5), (12, 16, 10), (3, 4, 7), (2, 2, 2), (16, 12, 33)]


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("dims", SMALL)
def test_project_fp64_small(bc, dims):
    nx, ny, nz = dims
    spec = W.small_spec(nx, ny, nz, bc[0], bc[1], lx=1.3, ly=0.9, lz=2.0, stretch=2.0)
    g = grid_of(spec)
    u, v, w = W.random_velocity(spec, nx * 7 + ny * 3 + nz)
    ru, rv, rw, rp = oracle.project(u, v, w, g, dt=0.37)
    gu, gv, gw, gp, info = run_project(spec, u, v, w, dt=0.37)
    print(f"dims={dims} bc={bc} errs u={rel(gu, ru):.2e} v={rel(gv, rv):.2e} w={rel(gw, rw):.2e} p={rel(gp, rp):.2e}")
    for a, b in ((gu, ru), (gv, rv), (gw, rw), (gp, rp)):
        assert rel(a, b) <= 1e-12
    assert abs(info["rhs_vmean_removed"]) < 1e-10


@pytest.mark.parametrize("dims,bc", [((96, 24, 50), (PERIODIC, WALL)), ((768, 6, 20), (WALL, PERIODIC)),
                                     ((6, 768, 12), (PERIODIC, WALL)), ((48, 96, 130), (WALL, WALL)),
                                     ((64, 32, 1000), (WALL, WALL))])
def test_project_fp64_tiles_and_ragged(dims, bc):
    """Several workgroup tiles per axis, radix-3 lengths, ragged z chunks."""
    nx, ny, nz = dims
    spec = W.small_spec(nx, ny, nz, bc[0], bc[1], lx=4.0, ly=4.0, lz=6.5, stretch=2.5)
    g = grid_of(spec)
    u, v, w = W.random_velocity(spec, 5)
    ru, rv, rw, rp = oracle.project(u, v, w, g)
    gu, gv, gw, gp, _ = run_project(spec, u, v, w)
    print(f"dims={dims} errs u={rel(gu, ru):.2e} v={rel(gv, rv):.2e} w={rel(gw, rw):.2e} p={rel(gp, rp):.2e}")
    for a, b in ((gu, ru), (gv, rv), (gw, rw), (gp, rp)):
        assert rel(a, b) <= 1e-12


@pytest.mark.parametrize("dims,bc", [((64, 192, 768), (WALL, WALL)), ((32, 288, 768), (PERIODIC, PERIODIC))])
def test_project_fp64_persistent_z_tiles(dims, bc):
    """768-row z lines in whole 32-mode tiles take the persistent z kernel
    (next tile's first rows staged in LDS); 384 and 288 tiles over at most
    one workgroup per CU, so workgroups solve several tiles in turn."""
    nx, ny, nz = dims
    spec = W.small_spec(nx, ny, nz, bc[0], bc[1], lx=4.0, ly=4.0, lz=6.5, stretch=2.5)
    g = grid_of(spec)
    u, v, w = W.random_velocity(spec, 11)
    ru, rv, rw, rp = oracle.project(u, v, w, g)
    gu, gv, gw, gp, _ = run_project(spec, u, v, w)
    print(f"dims={dims} errs u={rel(gu, ru):.2e} v={rel(gv, rv):.2e} w={rel(gw, rw):.2e} p={rel(gp, rp):.2e}")
    for a, b in ((gu, ru), (gv, rv), (gw, rw), (gp, rp)):
        assert rel(a, b) <= 1e-12


def test_project_fp64_c1():
    spec = W.CONFIGS["C1"]
    g = grid_of(spec)
    u, v, w = W.random_velocity(spec, W.SEEDS["C1"])
    ru, rv, rw, rp = oracle.project(u, v, w, g)
    gu, gv, gw, gp, _ = run_project(spec, u, v, w)
    errs = [rel(a, b) for a, b in ((gu, ru), (gv, rv), (gw, rw), (gp, rp))]
    print("C1 errs", errs)
    assert max(errs) <= 1e-12
    div = oracle.divergence(gu, gv, gw, g)
    assert np.abs(div).max() <= 1e-10 * np.abs(oracle.divergence(u, v, w, g)).max()


@pytest.mark.parametrize("bc", BCS)
def test_poisson_solve_incompatible_rhs_and_in_place(bc):
    F = fsei()
    spec = W.small_spec(24, 18, 28, bc[0], bc[1], lx=2.0, ly=1.5, lz=3.0, stretch=2.0)
    g = grid_of(spec)
    f = W.rng(3).standard_normal(spec.shape) + 0.25
    rp, rinfo = oracle.poisson_solve(f, g, return_info=True)
    plan = F.Plan.from_spec(spec)
    fd = dev(f)
    p, info = plan.poisson_solve(fd, info=True)
    assert rel(host(p), rp) <= 1e-12
    assert abs(info["rhs_vmean_removed"] - rinfo["rhs_vmean_removed"]) <= 1e-12
    plan.poisson_solve(fd, fd)                          # p aliases f
    torch.cuda.synchronize()
    assert rel(host(fd), rp) <= 1e-12


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("with_gp", [False, True])
def test_backward_fp64_matches_oracle_adjoint(bc, with_gp):
    F = fsei()
    spec = W.small_spec(12, 9, 14, bc[0], bc[1], lx=2.0, ly=1.5, lz=3.0, stretch=2.0)
    g = grid_of(spec)
    r = W.rng(17)
    gu, gv, gw = (r.standard_normal(spec.shape) for _ in range(3))
    gp = r.standard_normal(spec.shape) if with_gp else None
    mu, mv, mw = W.dead_face_masks(spec)
    gu[mu] = 0
    gv[mv] = 0
    gw[mw] = 0
    ref = oracle.project_adjoint(gu, gv, gw, gp, g, dt=0.6)
    plan = F.Plan.from_spec(spec)
    a, b, c = dev(gu), dev(gv), dev(gw)
    plan.project_backward(a, b, c, None if gp is None else dev(gp), dt=0.6)
    torch.cuda.synchronize()
    for x, y in zip((host(a), host(b), host(c)), ref):
        assert rel(x, y) <= 1e-12


def test_adjoint_dot_product_identity_c4a_shape():
    """<P x, y> = <x, P^T y> on the GPU alone at the C4a shape."""
    F = fsei()
    spec = W.CONFIGS["C4a"]
    plan = F.Plan.from_spec(spec)
    r = W.rng(44)
    x = [r.standard_normal(spec.shape) for _ in range(3)]
    y = [r.standard_normal(spec.shape) for _ in range(3)]
    for arrs in (x, y):
        for a, m in zip(arrs, W.dead_face_masks(spec)):
            a[m] = 0
    xd = [dev(a) for a in x]
    yd = [dev(a) for a in y]
    plan.project(*xd, dt=1.0, want_p=False)
    plan.project_backward(*yd, dt=1.0)
    torch.cuda.synchronize()
    lhs = sum(float((host(a) * b).sum()) for a, b in zip(xd, y))
    rhs = sum(float((a * host(b)).sum()) for a, b in zip(x, yd))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0) * 100


def test_gradcheck_tiny():
    F = fsei()
    spec = W.small_spec(4, 4, 6, PERIODIC, WALL, stretch=2.0)
    plan = F.Plan.from_spec(spec)
    r = W.rng(5)
    u, v, w = (dev(a) for a in W.random_velocity(spec, 5))
    wts = [dev(r.uniform(0.5, 1.5, spec.shape)) for _ in range(4)]

    def loss(a, b, c):
        uo, vo, wo, p = F.project(a, b, c, plan, dt=0.5)
        return (wts[0] * uo * uo).sum() + (wts[1] * vo * vo).sum() + (wts[2] * wo * wo).sum() + (wts[3] * p).sum()

    for t in (u, v, w):
        t.requires_grad_(True)
    mu, mv, mw = W.dead_face_masks(spec)
    # dead faces do not influence the outputs; perturb only active ones
    assert torch.autograd.gradcheck(loss, (u, v, w), eps=1e-6, atol=1e-8, rtol=1e-6, fast_mode=False,
                                    nondet_tol=1e-12)


def test_project_fp32_c1():
    F = fsei()
    spec = W.CONFIGS["C1"]
    g = grid_of(spec)
    u, v, w = W.random_velocity(spec, W.SEEDS["C1"])
    ru, rv, rw, rp = oracle.project(u, v, w, g)
    gu, gv, gw, gp, _ = run_project(spec, u, v, w, precision=F.PREC_FP32)
    errs = [rel(a, b) for a, b in ((gu, ru), (gv, rv), (gw, rw), (gp, rp))]
    print("C1 fp32 errs", errs)
    assert max(errs) <= 2e-5


@pytest.mark.parametrize("bc", [(WALL, WALL), (PERIODIC, WALL)])
def test_refine_projection_reaches_fp64(bc):
    F = fsei()
    spec = W.small_spec(64, 48, 96, bc[0], bc[1], lx=4.0, ly=4.0, lz=6.5, stretch=2.5)
    g = grid_of(spec)
    u, v, w = W.random_velocity(spec, 9)
    ru, rv, rw, rp = oracle.project(u, v, w, g)
    gu, gv, gw, gp, info = run_project(spec, u, v, w, precision=F.PREC_FP32_REFINE, rtol=1e-10, max_iter=6)
    print("refine info", info, [rel(a, b) for a, b in ((gu, ru), (gv, rv), (gw, rw), (gp, rp))])
    assert info["rel_residual"] <= 1e-10
    f = oracle.divergence(u, v, w, g)
    assert oracle.rel_residual(f, gp, g) <= 1e-10
    # p's V-mean is pinned in FP64 by the first correction, so p matches the
    # oracle to the level of the residual, not to FP32 rounding of its mean
    assert abs(oracle.vmean(gp, g)) <= 1e-13 * np.abs(gp).max()
    assert rel(gp, rp) <= 1e-10
    assert max(rel(gu, ru), rel(gv, rv), rel(gw, rw)) <= 1e-9


def _lam_tables(n, d, bc):
    """Modified wavenumbers as the plan tabulates them: in long double,
    rounded once to double and to float."""
    pi = np.longdouble("3.14159265358979323846264338327950288")
    q = np.arange(n)
    m = (q if bc == WALL else np.minimum(q, n - q)).astype(np.longdouble)
    arg = pi * m / (2 * n) if bc == WALL else pi * m / n
    lam = -np.longdouble(4) / (np.longdouble(d) * np.longdouble(d)) * np.sin(arg) ** 2
    return lam.astype(np.float64), lam.astype(np.float32)


def _routing_edge_grid(nx, ny, nz, bc):
    """z faces of a tanh grid, scaled so that the threshold of the FP64
    line routing, 4 / (dz_min^2 (kappa* - 1)) with kappa* = 1e4, lies within
    FP32 rounding of |lambda_x + lambda_y| of mode (1, 0): a scale is searched
    for which the host's FP64 test and the same test evaluated in FP32 on the
    FP32 tables disagree on some mode."""
    base = W.small_spec(nx, ny, nz, bc[0], bc[1], lx=4.0, ly=4.0, lz=1.0, stretch=1.5)
    zc0 = base.zc()
    lx64, lx32 = _lam_tables(nx, base.dx, bc[0])
    ly64, ly32 = _lam_tables(ny, base.dy, bc[1])
    s64 = np.abs(ly64[:, None] + lx64[None, :])
    s32 = np.abs(ly32[:, None] + lx32[None, :])
    s64[0, 0] = s32[0, 0] = np.inf
    target = s64[0, 1]
    for k in range(1, 200):
        for sgn in (1, -1):
            delta = sgn * k * 2e-9
            dzmin0 = float(np.diff(zc0.astype(np.longdouble)).astype(np.float64).min())
            scale = np.sqrt(4.0 / (dzmin0 ** 2 * 9999.0) / (target * (1 + delta)))
            zc = zc0 * scale
            dzmin = float(np.diff(zc.astype(np.longdouble)).astype(np.float64).min())
            thr = 4.0 / (dzmin * dzmin * (1e4 - 1.0))
            host_fp64 = s64 < thr
            fp32 = s32 < np.float32(thr)
            if np.any(host_fp64 != fp32):
                return base, zc
    raise AssertionError("no scale puts the routing threshold within FP32 rounding of a mode")


@pytest.mark.parametrize("bc", [(WALL, WALL), (PERIODIC, WALL)])
def test_fp64_line_routing_at_threshold(bc):
    """A mode line whose |lambda_x + lambda_y| lies within FP32 rounding of
    the routing threshold is solved exactly once: by the near-singular line
    kernel if the host listed it, else by the tiled kernel (both decide in
    FP64), in every precision mode."""
    F = fsei()
    base, zc = _routing_edge_grid(32, 24, 48, bc)
    g = oracle.Grid(base.nx, base.ny, base.nz, base.bcx, base.bcy, base.dx, base.dy, zc)
    u, v, w = W.random_velocity(base, 29)
    ru, rv, rw, rp = oracle.project(u, v, w, g)
    for prec, kw in ((F.PREC_FP64, {}), (F.PREC_FP32, {}), (F.PREC_FP32_REFINE, dict(rtol=1e-10, max_iter=6))):
        plan = F.Plan(base.nx, base.ny, base.nz, (base.bcx, base.bcy), base.dx, base.dy, zc, precision=prec, **kw)
        dtype = torch.float32 if prec == F.PREC_FP32 else torch.float64
        ud, vd, wd = dev(u, dtype), dev(v, dtype), dev(w, dtype)
        pd, info = plan.project(ud, vd, wd, info=True)
        torch.cuda.synchronize()
        errs = [rel(host(a), b) for a, b in ((ud, ru), (vd, rv), (wd, rw), (pd, rp))]
        print("routing edge", bc, prec, info, errs)
        if prec == F.PREC_FP64:
            assert max(errs) <= 1e-12
        elif prec == F.PREC_FP32:
            assert max(errs) <= 1e-4
        else:
            assert info["rel_residual"] <= 1e-10 and errs[3] <= 1e-10


def test_refine_fixed_iterations_and_not_converged():
    F = fsei()
    spec = W.small_spec(32, 32, 48, WALL, WALL, lx=4.0, ly=4.0, lz=6.5, stretch=2.5)
    u, v, w = W.random_velocity(spec, 10)
    plan = F.Plan.from_spec(spec, precision=F.PREC_FP32_REFINE, rtol=1e-30, max_iter=1)
    with pytest.raises(F.FseiError) as e:
        plan.project(dev(u), dev(v), dev(w), info=True)
    assert e.value.status == -6
    plan0 = F.Plan.from_spec(spec, precision=F.PREC_FP32_REFINE, rtol=0.0, max_iter=2)
    _, info = plan0.project(dev(u), dev(v), dev(w), info=True)
    assert info["iterations"] == 2 and info["rel_residual"] < 1e-9


# ---- fixed-length transform kernels (compile-time length 512) --------------
# x kernels: nx = 512 with ny a multiple of the 8 rows of a tile; y kernels:
# ny = 512 with nx a multiple of the tile width (16 FP64 / 32 FP32 columns).
FIXED = [((512, 16, 6), (WALL, WALL)), ((512, 24, 5), (PERIODIC, PERIODIC)), ((512, 8, 7), (PERIODIC, WALL)),
         ((32, 512, 5), (WALL, WALL)), ((64, 512, 4), (PERIODIC, PERIODIC)), ((16, 512, 6), (WALL, PERIODIC)),
         ((512, 512, 2), (WALL, WALL)), ((512, 512, 3), (PERIODIC, WALL)),
         # several plane chunks of the fused x-inverse + gradient (16 planes
         # each, a ragged last one), one 8-row tile whose halo row wraps
         ((512, 16, 40), (PERIODIC, PERIODIC)), ((512, 8, 37), (WALL, WALL)), ((512, 24, 33), (WALL, PERIODIC))]


@pytest.mark.parametrize("dims,bc", FIXED)
def test_project_fp64_fixed_length(dims, bc):
    nx, ny, nz = dims
    spec = W.small_spec(nx, ny, nz, bc[0], bc[1], lx=4.0, ly=3.0, lz=6.5, stretch=2.5)
    g = grid_of(spec)
    u, v, w = W.random_velocity(spec, nx + 3 * ny + 7 * nz)
    ru, rv, rw, rp = oracle.project(u, v, w, g, dt=0.8)
    gu, gv, gw, gp, _ = run_project(spec, u, v, w, dt=0.8)
    errs = [rel(a, b) for a, b in ((gu, ru), (gv, rv), (gw, rw), (gp, rp))]
    print(f"dims={dims} bc={bc} errs", errs)
    assert max(errs) <= 1e-12


@pytest.mark.parametrize("dims,bc", [d for d in FIXED if d[0][0] == 512 and d[0][1] % 8 == 0])
def test_refine_projection_fixed_length(dims, bc):
    """nx = 512: the first correction, the gradient correction and the
    convergence check run as one pass (several plane chunks with a ragged
    last one, both halo rows of an 8-row tile wrapping in periodic y).  The
    residual it reports is the residual of the p it stores."""
    F = fsei()
    nx, ny, nz = dims
    spec = W.small_spec(nx, ny, nz, bc[0], bc[1], lx=4.0, ly=3.0, lz=6.5, stretch=2.5)
    g = grid_of(spec)
    u, v, w = W.random_velocity(spec, 5 * nx + ny + nz)
    ru, rv, rw, rp = oracle.project(u, v, w, g, dt=0.8)
    gu, gv, gw, gp, info = run_project(spec, u, v, w, dt=0.8, precision=F.PREC_FP32_REFINE, rtol=1e-10,
                                       max_iter=6)
    f = oracle.divergence(u, v, w, g) / 0.8
    res = oracle.rel_residual(f, gp, g)
    errs = [rel(a, b) for a, b in ((gu, ru), (gv, rv), (gw, rw), (gp, rp))]
    print(f"dims={dims} bc={bc} info={info} host residual {res:.3e} errs", errs)
    assert info["iterations"] >= 1 and info["rel_residual"] <= 1e-10
    assert abs(info["rel_residual"] - res) <= 0.05 * res
    assert abs(oracle.vmean(gp, g)) <= 1e-13 * np.abs(gp).max()
    assert errs[3] <= 1e-10 and max(errs[:3]) <= 1e-9


def test_project_fp64_fixed_length_without_p():
    """u, v, w only (no pressure output): the fused x-inverse + gradient then
    writes no p at all."""
    F = fsei()
    spec = W.small_spec(512, 16, 40, WALL, PERIODIC, lx=4.0, ly=3.0, lz=6.5, stretch=2.5)
    g = grid_of(spec)
    u, v, w = W.random_velocity(spec, 77)
    ru, rv, rw, _ = oracle.project(u, v, w, g, dt=0.5)
    plan = F.Plan.from_spec(spec)
    ud, vd, wd = dev(u), dev(v), dev(w)
    assert plan.project(ud, vd, wd, dt=0.5, want_p=False) is None
    torch.cuda.synchronize()
    errs = [rel(host(a), b) for a, b in ((ud, ru), (vd, rv), (wd, rw))]
    print("without p", errs)
    assert max(errs) <= 1e-12


@pytest.mark.parametrize("dims,bc", [((512, 16, 6), (PERIODIC, WALL)), ((32, 512, 4), (WALL, PERIODIC)),
                                     ((512, 512, 2), (WALL, WALL)), ((512, 16, 40), (WALL, WALL)),
                                     ((512, 8, 37), (PERIODIC, PERIODIC))])
def test_backward_fp64_fixed_length(dims, bc):
    F = fsei()
    spec = W.small_spec(*dims, bc[0], bc[1], lx=2.0, ly=1.5, lz=3.0, stretch=2.0)
    g = grid_of(spec)
    r = W.rng(23)
    gu, gv, gw, gp = (r.standard_normal(spec.shape) for _ in range(4))
    for a, m in zip((gu, gv, gw), W.dead_face_masks(spec)):
        a[m] = 0
    ref = oracle.project_adjoint(gu, gv, gw, gp, g, dt=0.6)
    plan = F.Plan.from_spec(spec)
    a, b, c = dev(gu), dev(gv), dev(gw)
    plan.project_backward(a, b, c, dev(gp), dt=0.6)
    torch.cuda.synchronize()
    for x, y in zip((host(a), host(b), host(c)), ref):
        assert rel(x, y) <= 1e-12


@pytest.mark.parametrize("dims,bc", [((512, 8, 4), (WALL, WALL)), ((32, 512, 3), (PERIODIC, PERIODIC))])
def test_poisson_solve_fixed_length(dims, bc):
    F = fsei()
    spec = W.small_spec(*dims, bc[0], bc[1], lx=2.0, ly=1.5, lz=3.0, stretch=2.0)
    g = grid_of(spec)
    f = W.rng(31).standard_normal(spec.shape)
    rp = oracle.poisson_solve(f, g)
    p = F.Plan.from_spec(spec).poisson_solve(dev(f))
    torch.cuda.synchronize()
    assert rel(host(p), rp) <= 1e-12


@pytest.mark.parametrize("dims,bc", [((512, 32, 12), (WALL, WALL)), ((64, 512, 10), (PERIODIC, WALL)),
                                     ((512, 512, 4), (PERIODIC, PERIODIC))])
def test_fp32_and_refine_fixed_length(dims, bc):
    F = fsei()
    spec = W.small_spec(*dims, bc[0], bc[1], lx=4.0, ly=4.0, lz=6.5, stretch=2.5)
    g = grid_of(spec)
    u, v, w = W.random_velocity(spec, 77)
    ru, rv, rw, rp = oracle.project(u, v, w, g)
    fu, fv, fw, fp, _ = run_project(spec, u, v, w, precision=F.PREC_FP32)
    e32 = max(rel(a, b) for a, b in ((fu, ru), (fv, rv), (fw, rw)))
    gu, gv, gw, gp, info = run_project(spec, u, v, w, precision=F.PREC_FP32_REFINE, rtol=1e-10, max_iter=6)
    print(f"dims={dims} fp32 velocity err {e32:.2e} refine info {info}")
    assert e32 <= 2e-5
    assert info["rel_residual"] <= 1e-10
    assert oracle.rel_residual(oracle.divergence(u, v, w, g), gp, g) <= 1e-10
    assert max(rel(gu, ru), rel(gv, rv), rel(gw, rw)) <= 1e-9
    assert abs(oracle.vmean(gp, g)) <= 1e-13 * np.abs(gp).max() and rel(gp, rp) <= 1e-10


@pytest.mark.parametrize("rtol", [1e-10, 1e-13])
def test_refine_poisson_solve_reports_the_residual_of_its_result(rtol):
    """Solves take one residual pass per correction: the pass that prepares
    the next correction also gives the previous iterate's norm.  The reported
    residual is the one of the returned p (host check), for one correction
    and for several (rtol 1e-13, stopped at the FP64 floor or after four)."""
    F = fsei()
    spec = W.small_spec(64, 48, 96, WALL, PERIODIC, lx=4.0, ly=4.0, lz=6.5, stretch=2.5)
    g = grid_of(spec)
    f = W.rng(41).standard_normal(spec.shape)
    rp = oracle.poisson_solve(f, g)
    plan = F.Plan.from_spec(spec, precision=F.PREC_FP32_REFINE, rtol=rtol, max_iter=4, accept_floor=True)
    p, info = plan.poisson_solve(dev(f), info=True)
    torch.cuda.synchronize()
    gp = host(p)
    res = oracle.rel_residual(f, gp, g)
    print(f"rtol {rtol:.0e} info {info} host residual {res:.3e} p err {rel(gp, rp):.2e}")
    assert info["iterations"] >= (1 if rtol >= 1e-10 else 2)
    assert abs(info["rel_residual"] - res) <= 0.05 * res
    assert res <= max(rtol, 1e-12) or info["floor_reached"]
    assert rel(gp, rp) <= 1e-10


def test_refine_without_corrections_returns_the_fp32_solve():
    """max_iter = 0: the FP32 first solve, widened to FP64; its residual is
    the one the library reports."""
    F = fsei()
    spec = W.small_spec(64, 48, 96, WALL, WALL, lx=4.0, ly=4.0, lz=6.5, stretch=2.5)
    g = grid_of(spec)
    u, v, w = W.random_velocity(spec, 12)
    ru, rv, rw, rp = oracle.project(u, v, w, g)
    gu, gv, gw, gp, info = run_project(spec, u, v, w, precision=F.PREC_FP32_REFINE, rtol=0.0, max_iter=0)
    f = oracle.divergence(u, v, w, g)
    res = oracle.rel_residual(f, gp, g)
    print("no-correction info", info, "host residual", res, "p err", rel(gp, rp))
    assert info["iterations"] == 0
    assert abs(info["rel_residual"] - res) <= 0.05 * res
    assert rel(gp, rp) <= 1e-4 and max(rel(gu, ru), rel(gv, rv), rel(gw, rw)) <= 2e-5


def test_refine_projection_two_corrections():
    """rtol below what one correction reaches: the second correction adds to
    the FP64 iterate written by the first."""
    F = fsei()
    spec = W.small_spec(512, 32, 12, WALL, WALL, lx=4.0, ly=4.0, lz=6.5, stretch=2.5)
    g = grid_of(spec)
    u, v, w = W.random_velocity(spec, 77)
    ru, rv, rw, rp = oracle.project(u, v, w, g)
    gu, gv, gw, gp, info = run_project(spec, u, v, w, precision=F.PREC_FP32_REFINE, rtol=1e-13, max_iter=4)
    f = oracle.divergence(u, v, w, g)
    print("two-correction info", info)
    assert info["iterations"] == 2 and info["rel_residual"] <= 1e-13
    assert oracle.rel_residual(f, gp, g) <= 1e-13
    assert max(rel(gu, ru), rel(gv, rv), rel(gw, rw)) <= 1e-11


@pytest.mark.parametrize("dims,bc", [((27, 18, 40), (WALL, PERIODIC)), ((64, 36, 50), (PERIODIC, WALL)),
                                     ((64, 54, 96), (WALL, WALL)), ((81, 48, 40), (WALL, WALL))])
def test_refine_projection_generic_tiling(dims, bc):
    """Shapes outside the pair tiling (odd nx, or ny not a multiple of 8): the
    residual is the x-forward kernel's prologue (whose third partial sum
    carries the V-integral of p that the first correction removes) and the
    FP64 iterate is written by the first solve directly."""
    F = fsei()
    spec = W.small_spec(*dims, bc[0], bc[1], lx=4.0, ly=4.0, lz=6.5, stretch=2.5)
    g = grid_of(spec)
    u, v, w = W.random_velocity(spec, 21)
    ru, rv, rw, rp = oracle.project(u, v, w, g)
    gu, gv, gw, gp, info = run_project(spec, u, v, w, precision=F.PREC_FP32_REFINE, rtol=1e-10, max_iter=6)
    print("generic-tiling refine info", info, "p err", rel(gp, rp), "V-mean", oracle.vmean(gp, g))
    assert info["rel_residual"] <= 1e-10
    assert oracle.rel_residual(oracle.divergence(u, v, w, g), gp, g) <= 1e-10
    assert max(rel(gu, ru), rel(gv, rv), rel(gw, rw)) <= 1e-9
    assert abs(oracle.vmean(gp, g)) <= 1e-13 * np.abs(gp).max()
    assert rel(gp, rp) <= 1e-10


def test_long_z_lines_adjoint_fp32_and_refine():
    """nz = 1000: FP32 solves take the z tiling of 64 chunks of 16 rows, FP64
    ones 32 chunks of 32 rows with one mode per lane (two modes per lane
    would spill registers): the FP32 projection, FP32+refine and the FP64
    adjoint (transposed tridiagonal) against the oracle."""
    F = fsei()
    spec = W.small_spec(32, 16, 1000, PERIODIC, WALL, lx=4.0, ly=4.0, lz=6.5, stretch=3.0)
    g = grid_of(spec)
    u, v, w = W.random_velocity(spec, 31)
    ru, rv, rw, rp = oracle.project(u, v, w, g)
    gu, gv, gw, gp, _ = run_project(spec, u, v, w, precision=F.PREC_FP32)
    print("nz=1000 fp32 errs", [rel(a, b) for a, b in ((gu, ru), (gv, rv), (gw, rw), (gp, rp))])
    assert max(rel(a, b) for a, b in ((gu, ru), (gv, rv), (gw, rw), (gp, rp))) <= 1e-3   # a wrong tiling is O(1)
    gu, gv, gw, gp, info = run_project(spec, u, v, w, precision=F.PREC_FP32_REFINE, rtol=1e-9, max_iter=6)
    print("nz=1000 refine", info)
    assert info["rel_residual"] <= 1e-9
    assert max(rel(gu, ru), rel(gv, rv), rel(gw, rw)) <= 1e-8
    r = W.rng(32)
    au, av, aw = (r.standard_normal(spec.shape) for _ in range(3))
    for a, m in zip((au, av, aw), W.dead_face_masks(spec)):
        a[m] = 0
    ref = oracle.project_adjoint(au, av, aw, None, g, dt=0.6)
    plan = F.Plan.from_spec(spec)
    da, db, dc = dev(au), dev(av), dev(aw)
    plan.project_backward(da, db, dc, dt=0.6)
    torch.cuda.synchronize()
    errs = [rel(host(t), x) for t, x in zip((da, db, dc), ref)]
    print("nz=1000 adjoint errs", errs)
    assert max(errs) <= 1e-12


# ---- compile-time length 768 (x: tiles of 8 rows on 384 lanes; y: tiles of
# 128-byte row segments; the fused x-inverse + gradient at 768) -------------
L768 = [((768, 8, 12), (WALL, WALL)), ((768, 16, 20), (PERIODIC, WALL)), ((768, 24, 8), (WALL, PERIODIC)),
        ((16, 768, 8), (WALL, PERIODIC)), ((32, 768, 6), (PERIODIC, PERIODIC)), ((24, 768, 5), (WALL, WALL))]


def _check_all_precisions(spec, seed, bar32=2e-5):
    """FP64 projection, plain FP32, FP32+refine (residual, p and V-mean) and
    the FP64 adjoint of one shape against the oracle.  The FP64 bar is 1e-12,
    or three times the oracle's own error against its long-double variant on
    the same input where that floor is higher (white-noise input on lines of
    768-2048 points: up to ~3e-12 for the velocity component along the long
    line and for p on long z lines); the adjoint's the same way from the
    oracle's adjoint in long double."""
    F = fsei()
    g = grid_of(spec)
    u, v, w = W.random_velocity(spec, seed)
    ru, rv, rw, rp = oracle.project(u, v, w, g)
    ld = oracle.project(u, v, w, g, dtype=np.longdouble)
    floor = max(rel(a, np.asarray(b, dtype=np.float64)) for a, b in zip((ru, rv, rw, rp), ld))
    bar64 = max(1e-12, 3.0 * floor)
    out = run_project(spec, u, v, w)
    e64 = [rel(a, b) for a, b in zip(out[:4], (ru, rv, rw, rp))]
    out = run_project(spec, u, v, w, precision=F.PREC_FP32)
    e32 = [rel(a, b) for a, b in zip(out[:4], (ru, rv, rw, rp))]
    # refinement to 1e-12 (two corrections, or the FP64 floor of the input):
    # one correction to 1e-10 leaves forward errors up to ~1e-9 on these
    # lines, two bring them to the FP64 level
    gu, gv, gw, gp, info = run_project(spec, u, v, w, precision=F.PREC_FP32_REFINE, rtol=1e-12, max_iter=6,
                                       accept_floor=True)
    er = [rel(a, b) for a, b in zip((gu, gv, gw, gp), (ru, rv, rw, rp))]
    r = W.rng(seed + 1)
    au, av, aw, ap = (r.standard_normal(spec.shape) for _ in range(4))
    for a, m in zip((au, av, aw), W.dead_face_masks(spec)):
        a[m] = 0
    ref = oracle.project_adjoint(au, av, aw, ap, g, dt=0.6)
    ref_ld = oracle.project_adjoint(au, av, aw, ap, g, dt=0.6, dtype=np.longdouble)
    floor_adj = max(rel(a, np.asarray(b, dtype=np.float64)) for a, b in zip(ref, ref_ld))
    bar_adj = max(1e-12, 3.0 * floor_adj)
    plan = F.Plan.from_spec(spec)
    da, db, dc = dev(au), dev(av), dev(aw)
    plan.project_backward(da, db, dc, dev(ap), dt=0.6)
    torch.cuda.synchronize()
    ea = [rel(host(t), x) for t, x in zip((da, db, dc), ref)]
    print(f"{(spec.nx, spec.ny, spec.nz)} fp64 {max(e64):.2e} (oracle floor {floor:.2e}) fp32 {max(e32):.2e} "
          f"refine {info} {max(er):.2e} adjoint {max(ea):.2e} (floor {floor_adj:.2e})")
    assert max(e64) <= bar64
    assert max(e32) <= bar32
    assert info["rel_residual"] <= (1e-10 if info["floor_reached"] else 1e-12)
    assert max(er) <= max(1e-10, 30.0 * floor)
    # the first correction pins the V-mean of p in FP64 up to the FP32
    # rounding of the correction itself (about eps32 times its size, which
    # is the plain FP32 error of p)
    assert abs(oracle.vmean(gp, g)) <= max(1e-13, 10 * 2.0 ** -24 * max(e32)) * np.abs(gp).max()
    assert max(ea) <= bar_adj


@pytest.mark.parametrize("ny", [256, 96])
def test_persistent_z_tiles_fp32_and_refine(ny):
    """768-row z lines in whole 64-mode tiles: 256 of them (more than the
    persistent FP32 z kernel has workgroups) and 96 (fewer: one tile per
    workgroup); plain FP32 and FP32+refine against the FP64 oracle (bars as
    for the fixed-length shapes, plain FP32 at 5e-5 for 768-point lines)."""
    F = fsei()
    spec = W.small_spec(64, ny, 768, WALL, PERIODIC, lx=4.0, ly=4.0, lz=6.5, stretch=2.0)
    g = grid_of(spec)
    u, v, w = W.random_velocity(spec, 29)
    ru, rv, rw, rp = oracle.project(u, v, w, g)
    fu, fv, fw, fp, _ = run_project(spec, u, v, w, precision=F.PREC_FP32)
    e32 = max(rel(a, b) for a, b in ((fu, ru), (fv, rv), (fw, rw)))
    # rtol 1e-12: the error of p follows the residual times the condition of
    # the lowest modes (residual 1.3e-11 left p at 1.1e-10 on the 96-row shape)
    gu, gv, gw, gp, info = run_project(spec, u, v, w, precision=F.PREC_FP32_REFINE, rtol=1e-12, max_iter=6)
    print(f"fp32 velocity err {e32:.2e} refine info {info}")
    assert e32 <= 5e-5
    assert info["rel_residual"] <= (1e-10 if info["floor_reached"] else 1e-12)
    assert oracle.rel_residual(oracle.divergence(u, v, w, g), gp, g) <= 1e-10
    assert max(rel(gu, ru), rel(gv, rv), rel(gw, rw)) <= 1e-9
    assert abs(oracle.vmean(gp, g)) <= 1e-13 * np.abs(gp).max() and rel(gp, rp) <= 1e-10


@pytest.mark.parametrize("dims,bc", L768)
def test_length_768_all_precisions(dims, bc):
    """Plain FP32 at 5e-5: its rounding grows with the transform length
    (about eps32 per radix stage and pre/post pass, 4 + 2 passes per
    direction at 768 against 3 + 2 at 512 and 2 + 2 at 64) and with the
    condition of the mode lines kept in FP32 (up to 1e4); measured
    1.3e-5 to 2.1e-5 at 768, against 2e-5 at 64^3."""
    spec = W.small_spec(*dims, bc[0], bc[1], lx=4.0, ly=4.0, lz=6.5, stretch=2.0)
    _check_all_precisions(spec, sum(dims), bar32=5e-5)


@pytest.mark.parametrize("dims,bc", [((1536, 8, 4), (WALL, PERIODIC)), ((8, 2048, 4), (PERIODIC, WALL)),
                                     ((16, 8, 1536), (WALL, WALL)), ((16, 8, 2048), (PERIODIC, WALL)),
                                     ((18, 8, 2048), (WALL, WALL))])
def test_longest_lines_all_precisions(dims, bc):
    """The longest accepted lines: x and y transforms of one sequence per
    tile (1536, 2048), z lines of up to 64 chunks (1536, 2048 rows; nx = 18
    is not a multiple of 4: two FP32 modes per lane)."""
    spec = W.small_spec(*dims, bc[0], bc[1], lx=4.0, ly=4.0, lz=6.5, stretch=2.0)
    # plain FP32 on lines of 1536-2048 points: rounding of the longer
    # transform chains (measured up to 5.6e-5 at nx = 1536) and, on long z
    # lines, mode lines kept in FP32 up to the routing threshold 1e4; the
    # bars are set for what plain FP32 is checked for here, the tilings and
    # chunk joins of these lengths, whose mistakes give O(1) errors (FP64
    # and the refinement keep their strict bars)
    _check_all_precisions(spec, 3 * sum(dims), bar32=1e-3 if spec.nz > 1024 else 2e-4)
