"""Point evaluation, adjoint and Newton projection on the GPU.

* values: bit-identical to the oracle's round-to-nearest nested Horner;
* Jacobian: the oracle's derivative polynomials (coefficients e_j c_e),
  within the Horner error bound, and central finite differences;
* coefficient adjoint on a CSF grid of centres: exact rational sums;
* Newton projection onto sphere ∩ plane converges to the exact circle;
* the torch.autograd.Function passes gradcheck.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import core as orc
from paper_2406_09857_amd import synth
from tests.helpers import bits_equal

pytestmark = pytest.mark.gpu
EPS = 2.0 ** -53


@pytest.fixture(scope="module")
def vx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_09857_amd import binding
    binding.lib()
    return binding


def deriv_cube(c, j):
    """Coefficients of dF/dx_j: e_j c_e moved to exponent e - u_j (rounded to nearest)."""
    k = c.ndim
    e = np.indices(c.shape)[j].astype(np.float64)
    d = c * e
    sl = [slice(None)] * k
    sl[j] = slice(1, None)
    out = np.zeros_like(c)
    osl = [slice(None)] * k
    osl[j] = slice(0, c.shape[j] - 1)
    out[tuple(osl)] = d[tuple(sl)]
    return out


def horner_bound(c, dgr, x):
    """gamma_{4d} * |P|(|x|): error bound of a nested Horner evaluation."""
    absv = orc.eval_points(np.abs(c), dgr, np.abs(x))
    return 4 * (4 * dgr + 8) * EPS * absv


@pytest.mark.parametrize("k,d", [(1, 30), (2, 20), (3, 12), (4, 6), (3, 100)])
def test_values_bitexact_and_jacobian(vx, k, d):
    import torch
    print(f"[grad] k={k} d={d}", flush=True)
    rng = np.random.default_rng(1000 + k * 10 + d)
    polys = synth.small_random(k, d, seed=1100 + d, npolys=2)
    x = rng.uniform(-1, 1, size=(777 if d < 100 else 200, k))
    f, jac, _, _ = vx.eval_grad(polys, torch.as_tensor(x, device="cuda"))
    f = f.cpu().numpy(); jac = jac.cpu().numpy()
    for p, c in enumerate(polys):
        ref = orc.eval_points(c, d, x)
        assert bits_equal(f[p], ref)
        for j in range(k):
            dc = deriv_cube(c, j)
            dref = orc.eval_points(dc, d, x)
            tol = horner_bound(dc, d, x) + horner_bound(c, d, x) * d
            assert np.all(np.abs(jac[:, p, j] - dref) <= tol + 1e-300), (p, j)


def test_jacobian_central_differences(vx):
    import torch
    rng = np.random.default_rng(5)
    w = synth.tiny()
    c = w.polys[0] / 100.0
    x = rng.uniform(-0.8, 0.8, size=(500, 2))
    h = 1e-6
    _, jac, _, _ = vx.eval_grad([c], torch.as_tensor(x, device="cuda"))
    jac = jac.cpu().numpy()[:, 0, :]
    for j in range(2):
        xp = x.copy(); xp[:, j] += h
        xm = x.copy(); xm[:, j] -= h
        fp = vx.eval_grad([c], torch.as_tensor(xp, device="cuda"), want_jac=False)[0].cpu().numpy()[0]
        fm = vx.eval_grad([c], torch.as_tensor(xm, device="cuda"), want_jac=False)[0].cpu().numpy()[0]
        fd = (fp - fm) / (2 * h)
        rel = np.abs(fd - jac[:, j]) / np.maximum(np.abs(jac).max(axis=1), 1e-30)
        assert np.max(rel) <= 1e-7, np.max(rel)


def _grid(level, k, n, seed):
    rng = np.random.default_rng(seed)
    return orc.csf_from_boxes(rng.integers(0, 1 << level, size=(n, k)), level)


@pytest.mark.parametrize("k,d,level,n,seed", [(3, 5, 3, 150, 11), (1, 9, 7, 100, 21), (2, 7, 6, 300, 31),
                                              (4, 3, 2, 120, 41)])
def test_coefficient_adjoint_exact(vx, k, d, level, n, seed):
    """dF/dcoef on a CSF grid of centres against exact rational sums, for
    every k: the root's children and the parents of the leaves come in
    chunks of 32 with short input rows staged on the device (more than 32
    children at the root for k = 1 and 2)."""
    import torch
    print(f"[adjoint] k={k} d={d} level={level}", flush=True)
    S = _grid(level, k, n, seed)
    c = synth.small_random(k, d, seed=seed + 1)[0]
    dom = np.array([-1.0, 1.0] * k)
    csf = vx.CSF.from_arrays(k, level, S["idx"], S["ptr"])
    x = vx.csf_centres(csf, dom)
    xs = x.cpu().numpy()
    # centres are exact dyadics
    want = -1.0 + (2 * S["boxes"] + 1) / (1 << level)
    assert np.array_equal(xs, want)
    rng = np.random.default_rng(seed + 2)
    gbar = rng.standard_normal((1, xs.shape[0]))
    _, _, xbar, dcoef = vx.eval_grad([c], x, want_jac=True, gbar=torch.as_tensor(gbar, device="cuda"),
                                     want_xbar=True, want_dcoef=True, grid=csf, dom=dom)
    dcoef = dcoef.cpu().numpy()[0]
    fx = [[Fraction(float(v)) for v in row] for row in xs]
    fg = [Fraction(float(v)) for v in gbar[0]]
    def mono(fx_i, e):
        m = Fraction(1)
        for j in range(k):
            m *= fx_i[j] ** int(e[j])
        return m

    for e in np.argwhere(synth.simplex_mask(k, d)):
        ex = sum(g * mono(fx_i, e) for g, fx_i in zip(fg, fx))
        bound = sum(abs(g) * abs(mono(fx_i, e)) for g, fx_i in zip(fg, fx))
        tol = (len(fg) + k * d + 4) * EPS * float(bound)
        assert abs(float(Fraction(float(dcoef[tuple(e)])) - ex)) <= tol + 1e-300, tuple(e)
    outside = ~synth.simplex_mask(k, d)
    assert np.all(dcoef[outside] == 0.0)
    # xbar = gbar * dF/dx
    _, jac, _, _ = vx.eval_grad([c], x)
    assert np.allclose(xbar.cpu().numpy(), gbar[0][:, None] * jac.cpu().numpy()[:, 0, :], rtol=0, atol=0)


def test_coefficient_adjoint_curve_sample(vx):
    """Degree-100 curve polynomials on the kept centres of level 6 (oracle
    subdivision): sampled coefficients against long-double sums with bounds."""
    import torch
    w = synth.curve()
    rec = orc.subdivide(w.polys, 3, 6, nthreads=orc.max_threads())[-1]
    K = orc.csf_from_boxes(rec["kept"], 6)
    csf = vx.CSF.from_arrays(3, 6, K["idx"], K["ptr"])
    dom = w.domain()
    x = vx.csf_centres(csf, dom)
    rng = np.random.default_rng(21)
    gbar = rng.standard_normal((2, x.shape[0]))
    _, _, _, dcoef = vx.eval_grad(w.polys, x, want_jac=False, gbar=torch.as_tensor(gbar, device="cuda"),
                                  want_dcoef=True, grid=csf, dom=dom)
    dcoef = dcoef.cpu().numpy()
    xs = x.cpu().numpy().astype(np.longdouble)
    es = np.argwhere(synth.simplex_mask(3, 100))
    for e in es[rng.choice(len(es), 60, replace=False)]:
        mono = xs[:, 0] ** int(e[0]) * xs[:, 1] ** int(e[1]) * xs[:, 2] ** int(e[2])
        for p in range(2):
            ref = np.sum(gbar[p].astype(np.longdouble) * mono)
            bound = np.sum(np.abs(gbar[p]) * np.abs(mono))
            tol = (x.shape[0] + 310) * EPS * float(bound)
            assert abs(float(dcoef[p][tuple(e)]) - float(ref)) <= tol + 1e-300


def test_newton_projects_onto_sphere_plane_circle(vx):
    import torch
    polys = [synth.sphere(), synth.plane_x3()]
    recs = orc.subdivide(polys, 3, 5)
    K = orc.csf_from_boxes(recs[-1]["kept"], 5)
    csf = vx.CSF.from_arrays(3, 5, K["idx"], K["ptr"])
    x = vx.csf_centres(csf, np.array([-1.0, 1.0] * 3))
    f0 = vx.eval_grad(polys, x, want_jac=False)[0].abs().max().item()
    x, f = vx.newton_project(polys, x, steps=3)
    assert f0 > 1e-3 and f.abs().max().item() < 1e-9  # quadratic convergence from cells of width 1/16
    x, f = vx.newton_project(polys, x, steps=3)
    xs = x.cpu().numpy()
    assert f.abs().max().item() < 1e-14
    assert np.all(np.abs(xs[:, 2] - 1.0 / 3.0) < 1e-14)
    assert np.all(np.abs(xs[:, 0] ** 2 + xs[:, 1] ** 2 - (0.5 - (1.0 / 3.0) ** 2)) < 1e-14)


def test_newton_step_matches_cpu_on_curve(vx):
    """One minimum-norm Newton step from sampled level-5 kept centres of the
    degree-100 curve system, against the same step computed on the CPU from
    the oracle's values and derivative polynomials (points whose J J^T is
    well conditioned)."""
    import torch
    w = synth.curve()
    rec = orc.subdivide(w.polys, 3, 5, nthreads=orc.max_threads())[-1]
    rng = np.random.default_rng(41)
    kept = rec["kept"][rng.choice(len(rec["kept"]), 120, replace=False)]
    x0 = -1.0 + (2 * kept + 1) / 32.0
    x = torch.as_tensor(x0.copy(), device="cuda")
    x1, _ = vx.newton_project(w.polys, x, steps=1)
    step_gpu = x0 - x1.cpu().numpy()
    F = np.stack([orc.eval_points(c, 100, x0) for c in w.polys], 1)                     # n, 2
    J = np.stack([np.stack([orc.eval_points(deriv_cube(c, j), 100, x0) for j in range(3)], 1)
                  for c in w.polys], 1)                                                  # n, 2, 3
    JJt = J @ J.transpose(0, 2, 1)
    step_cpu = (J.transpose(0, 2, 1) @ np.linalg.solve(JJt, F[:, :, None]))[:, :, 0]
    cond = np.linalg.cond(JJt)
    ok = cond < 1e6
    assert ok.sum() >= 60
    err = np.linalg.norm(step_gpu - step_cpu, axis=1)[ok]
    ref = np.linalg.norm(step_cpu, axis=1)[ok]
    assert np.all(err <= 1e-7 * ref + 1e-13), np.max(err / np.maximum(ref, 1e-300))


def test_polyeval_gradcheck(vx):
    import torch
    from torch.autograd import gradcheck
    c1, c2 = (torch.as_tensor(c, device="cuda") for c in synth.small_random(3, 4, seed=31, npolys=2))
    rng = np.random.default_rng(32)
    x = torch.as_tensor(rng.uniform(-0.9, 0.9, size=(20, 3)), device="cuda").requires_grad_(True)
    assert gradcheck(lambda xx: vx.PolyEval.apply(xx, None, c1, c2), (x,), eps=1e-6, atol=1e-7, rtol=1e-6)
    # coefficient gradients on a grid of centres (the grid is an argument of the call)
    S = _grid(3, 3, 30, 33)
    csf = vx.CSF.from_arrays(3, 3, S["idx"], S["ptr"])
    dom = np.array([-1.0, 1.0] * 3)
    xg = vx.csf_centres(csf, dom)
    a = c1.clone().requires_grad_(True)
    b = c2.clone().requires_grad_(True)
    assert gradcheck(lambda p, q: vx.PolyEval.apply(xg, (csf, dom), p, q), (a, b), eps=1e-6, atol=1e-7, rtol=1e-6)
    # the grid forward equals the per-point forward bit for bit
    assert bits_equal(vx.PolyEval.apply(xg, (csf, dom), c1, c2).cpu().numpy(),
                      vx.PolyEval.apply(xg, None, c1, c2).cpu().numpy())


def test_grid_points_must_be_the_grid_centres(vx):
    """Points that are not, bit for bit, the centres of the grid's leaves (a
    stale grid, or points a Newton step moved) are refused, not silently
    evaluated at the centres."""
    import torch
    c = synth.small_random(3, 5, seed=34, npolys=1)
    S = _grid(3, 3, 40, 35)
    csf = vx.CSF.from_arrays(3, 3, S["idx"], S["ptr"])
    dom = np.array([-1.0, 1.0] * 3)
    xg = vx.csf_centres(csf, dom)
    vx.eval_grad(c, xg, grid=csf, dom=dom)  # the centres pass
    moved = xg.clone()
    moved[17, 1] += 1e-12
    with pytest.raises(vx.VxError, match="centres"):
        vx.eval_grad(c, moved, grid=csf, dom=dom)
    other = vx.CSF.from_arrays(3, 3, S["idx"], S["ptr"])
    with pytest.raises(vx.VxError, match="centres"):
        vx.eval_grad(c, vx.csf_centres(other, np.array([-1.0, 1.0, -1.0, 1.0, -1.0, 0.5])), grid=csf, dom=dom)
    with pytest.raises(vx.VxError, match="centres"):
        vx.PolyEval.apply(moved, (csf, dom), torch.as_tensor(c[0], device="cuda"))


@pytest.mark.parametrize("k,d,level,n", [(1, 40, 9, 300), (2, 20, 6, 900), (3, 12, 4, 700), (4, 6, 3, 500),
                                         (3, 100, 5, 400)])
def test_grid_forward_bit_identical_to_per_point(vx, k, d, level, n):
    """The amortized forward on a CSF grid (f and the Jacobian) equals the
    per-point evaluation bit for bit, and the values equal the oracle's
    round-to-nearest Horner, for k = 1..4, two polynomials, on a
    non-dyadic domain too."""
    import torch
    print(f"[grad] grid forward k={k} d={d} level={level}", flush=True)
    polys = synth.small_random(k, d, seed=1200 + k * 10 + d, npolys=2)
    for dom in (np.array([-1.0, 1.0] * k), np.array([-0.7, 1.3, -1.1, 0.9, -2.0, 0.25, -0.5, 0.5][: 2 * k])):
        S = _grid(level, k, n, 1300 + k)
        csf = vx.CSF.from_arrays(k, level, S["idx"], S["ptr"])
        x = vx.csf_centres(csf, dom)
        fg, jg, _, _ = vx.eval_grad(polys, None, grid=csf, dom=dom)
        fp, jp, _, _ = vx.eval_grad(polys, x)
        assert bits_equal(fg.cpu().numpy(), fp.cpu().numpy())
        assert bits_equal(jg.cpu().numpy(), jp.cpu().numpy())
        f1, _, _, _ = vx.eval_grad(polys, x, want_jac=False, grid=csf, dom=dom)
        assert bits_equal(f1.cpu().numpy(), fp.cpu().numpy())
        xs = x.cpu().numpy()
        for p, c in enumerate(polys):
            assert bits_equal(fg.cpu().numpy()[p], orc.eval_points(c, d, xs))


@pytest.mark.parametrize("k,d,level,n", [(2, 20, 6, 900), (3, 12, 4, 700), (3, 100, 5, 400)])
def test_newton_from_grid_bit_identical(vx, k, d, level, n):
    """newton_project_grid (first evaluation on the CSF grid of centres)
    gives the points and values of newton_project bit for bit, and refuses
    points that are not the grid's centres, leaving them unchanged."""
    import torch
    print(f"[newton-grid] k={k} d={d} level={level}", flush=True)
    polys = synth.small_random(k, d, seed=1300 + d, npolys=min(k, 2))
    S = _grid(level, k, n, 1310 + k)
    csf = vx.CSF.from_arrays(k, level, S["idx"], S["ptr"])
    dom = np.array([-0.7, 1.3] * k)
    x0 = vx.csf_centres(csf, dom)
    xa, fa = vx.newton_project(polys, x0.clone(), steps=3)
    xb, fb = vx.newton_project(polys, x0.clone(), steps=3, grid=(csf, dom))
    assert bits_equal(xa.cpu().numpy(), xb.cpu().numpy())
    assert bits_equal(fa.cpu().numpy(), fb.cpu().numpy())
    moved = x0.clone()
    moved[n // 2, 0] += 1e-12
    keep = moved.clone()
    with pytest.raises(vx.VxError, match="centres"):
        vx.newton_project(polys, moved, steps=3, grid=(csf, dom))
    assert torch.equal(moved, keep)
