"""Contract edges of the C ABI against the oracle (include/fsei.h): wall
faces are ignored on input and written 0 on output, in the projection and
in its adjoint, for every precision mode and for the fixed-length and generic
kernel paths; the adjoint and the autograd wrapper under FP32_REFINE plans
(the adjoint is computed in FP64 there).  FP64 bars: 1e-12, or three times
the oracle's own error against its long-double variant where that is higher
(768-point lines); plain FP32 5e-5 (as for the other 768-point tests)."""
import numpy as np
import pytest

import oracle
from oracle import PERIODIC, WALL
from paper_2103_15187_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def fsei():
    from paper_2103_15187_amd import fsei as F
    return F


def grid_of(spec):
    return oracle.Grid(spec.nx, spec.ny, spec.nz, spec.bcx, spec.bcy, spec.dx, spec.dy, spec.zc())


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def with_garbage(fields, spec, seed):
    """Copies of the fields with large values on every dead wall face."""
    r = W.rng(seed)
    out = []
    for a, m in zip(fields, W.dead_face_masks(spec)):
        b = a.copy()
        b[m] = 1e3 * r.standard_normal(int(m.sum()))
        out.append(b)
    return out


SHAPES = [((16, 12, 10), (WALL, WALL)), ((512, 16, 6), (WALL, WALL)), ((768, 8, 5), (WALL, PERIODIC)),
          ((24, 512, 4), (PERIODIC, WALL))]


@pytest.mark.parametrize("dims,bc", SHAPES)
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_refine"])
def test_projection_ignores_and_zeroes_dead_faces(dims, bc, prec):
    F = fsei()
    spec = W.small_spec(*dims, bc[0], bc[1], lx=4.0, ly=4.0, lz=6.5, stretch=2.5)
    g = grid_of(spec)
    clean = W.random_velocity(spec, 61)
    ref = oracle.project(*clean, g, dt=0.9)
    # FP64 bar: 1e-12, or 3x the oracle's own error against long double where
    # that floor is higher (lines of 768 points)
    ld = oracle.project(*clean, g, dt=0.9, dtype=np.longdouble)
    bar64 = max(1e-12, 3.0 * max(rel(a, np.asarray(b, dtype=np.float64)) for a, b in zip(ref, ld)))
    dirty = with_garbage(clean, spec, 62)
    kw = {"fp64": {}, "fp32": dict(precision=F.PREC_FP32),
          "fp32_refine": dict(precision=F.PREC_FP32_REFINE, rtol=1e-10, max_iter=6)}[prec]
    dtype = torch.float32 if prec == "fp32" else torch.float64
    plan = F.Plan.from_spec(spec, **kw)
    d = [dev(a, dtype) for a in dirty]
    p = plan.project(*d, dt=0.9)
    torch.cuda.synchronize()
    out = [t.double().cpu().numpy() for t in (*d, p)]
    errs = [rel(a, b) for a, b in zip(out, ref)]
    print(dims, bc, prec, errs)
    assert max(errs) <= {"fp64": bar64, "fp32": 5e-5, "fp32_refine": 1e-9}[prec]
    for a, m in zip(out[:3], W.dead_face_masks(spec)):
        assert np.all(a[m] == 0.0)


@pytest.mark.parametrize("dims,bc", SHAPES)
@pytest.mark.parametrize("prec", ["fp64", "fp32_refine"])
def test_adjoint_ignores_and_zeroes_dead_faces(dims, bc, prec):
    """g_u on dead faces multiplies outputs that are always 0, so it must not
    reach dLoss/du*; dLoss/du* on dead faces (inputs that are ignored) is 0.
    FP32_REFINE plans compute the adjoint in FP64."""
    F = fsei()
    spec = W.small_spec(*dims, bc[0], bc[1], lx=4.0, ly=4.0, lz=6.5, stretch=2.5)
    g = grid_of(spec)
    r = W.rng(63)
    gu, gv, gw, gp = (r.standard_normal(spec.shape) for _ in range(4))
    ref = oracle.project_adjoint(gu, gv, gw, gp, g, dt=0.7)
    ld = oracle.project_adjoint(gu, gv, gw, gp, g, dt=0.7, dtype=np.longdouble)
    bar = max(1e-12, 3.0 * max(rel(a, np.asarray(b, dtype=np.float64)) for a, b in zip(ref, ld)))
    kw = {} if prec == "fp64" else dict(precision=F.PREC_FP32_REFINE, rtol=1e-10, max_iter=4)
    plan = F.Plan.from_spec(spec, **kw)
    d = [dev(a) for a in with_garbage((gu, gv, gw), spec, 64)]
    plan.project_backward(*d, dev(gp), dt=0.7)
    torch.cuda.synchronize()
    out = [t.cpu().numpy() for t in d]
    errs = [rel(a, b) for a, b in zip(out, ref)]
    print(dims, bc, prec, errs)
    assert max(errs) <= bar
    for a, m in zip(out, W.dead_face_masks(spec)):
        assert np.all(a[m] == 0.0)


def test_autograd_under_refine_plan():
    """ProjectFn with an FP32_REFINE plan: the forward to the refinement's
    accuracy, the gradient of a weighted quadratic loss (its adjoint in FP64)
    against the oracle's W P W^-1 (omega * P u*)."""
    F = fsei()
    spec = W.small_spec(32, 24, 40, PERIODIC, WALL, lx=4.0, ly=4.0, lz=6.5, stretch=2.0)
    g = grid_of(spec)
    u, v, w = W.random_velocity(spec, 65)
    om = W.face_weights_random(spec, 66)
    pu, pv, pw, _ = oracle.project(u, v, w, g)
    ref = oracle.project_adjoint(om[0] * pu, om[1] * pv, om[2] * pw, None, g)
    plan = F.Plan.from_spec(spec, precision=F.PREC_FP32_REFINE, rtol=1e-12, max_iter=6)
    d = [dev(a).requires_grad_(True) for a in (u, v, w)]
    omd = [dev(a) for a in om]
    uo, vo, wo, _ = F.project(*d, plan)
    loss = 0.5 * sum((o * x * x).sum() for o, x in zip(omd, (uo, vo, wo)))
    loss.backward()
    fe = [rel(t.detach().cpu().numpy(), r_) for t, r_ in zip((uo, vo, wo), (pu, pv, pw))]
    ge = [rel(t.grad.cpu().numpy(), r_) for t, r_ in zip(d, ref)]
    print("refine autograd forward", fe, "gradient", ge)
    assert max(fe) <= 1e-10
    assert max(ge) <= 1e-10
