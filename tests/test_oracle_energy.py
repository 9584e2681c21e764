"""Pins of the energy-advection oracle (oracle/energy.py, Eq. energy_advection).

* the face reconstruction: exact on linear data (both candidate stencils
  agree), the smooth stencil chosen across a step (the ENO property of the
  nonlinear weights), and with the linear weights (eps -> infinity) the
  derivative exact for quadratics, which fixes d = (1/3, 2/3) and the
  candidates;
* the step is forward Euler: a linear field moves by exactly dt u . grad T
  in each phase, each cell with its own phase's field and velocity;
* the upwind side follows the sign of each velocity component: a step is
  carried one CFL fraction downstream either way and the upstream side
  stays put;
* the derivative converges at second order or better on smooth data (the
  nonlinear weights of the Jiang & Shu scheme are within O(h) of the linear
  ones);
* invariants of the stencil handling: shifting a periodic field shifts the
  result, mirroring the box and the flow mirrors it (walls clamp
  symmetrically); zero velocity or dt = 0 returns T unchanged.
"""
import numpy as np
import pytest

from energy_util import cell_centres, energy_case, face_velocities, rough_field, smooth_field
from oracle import energy


def test_face_exact_on_linear_data():
    rng = np.random.Generator(np.random.PCG64(1))
    a, b = rng.normal(size=(2, 100)) * 10.0
    got = energy.weno3_face(a - b, a, a + b)
    assert np.max(np.abs(got - (a + 0.5 * b))) <= 1e-13 * np.max(np.abs(a) + np.abs(b))


def test_face_takes_the_smooth_side_of_a_step():
    # (m, 0 | p): the jump between m and 0 -> the flat stencil (0, p);
    # between 0 and p -> the flat upwind stencil (m, 0)
    assert abs(energy.weno3_face(0.0, 1.0, 1.0) - 1.0) < 1e-11
    assert abs(energy.weno3_face(0.0, 0.0, 1.0) - 0.0) < 1e-11
    assert abs(energy.weno3_face(5.0, 2.0, 2.0) - 2.0) < 1e-10
    assert abs(energy.weno3_face(2.0, 2.0, -3.0) - 2.0) < 1e-10


@pytest.mark.parametrize("sign", [1, -1])
def test_linear_weights_differentiate_quadratics_exactly(sign):
    case = energy_case(2, (24, 8, 1), periodic=(False, True, False))
    x, y, _ = cell_centres(case)
    c = (0.3, -1.7, 2.5)
    T = c[0] + c[1] * x + c[2] * x ** 2 + 0.0 * y
    inner = np.nonzero((x > 2.5 * case.h) & (x < 1.0 - 2.5 * case.h))[0]
    d = energy.derivative(case, T, 0, sign, inner, eps=1e30)
    assert np.max(np.abs(d - (c[1] + 2 * c[2] * x[inner]))) < 1e-11
    # with the default eps the nonlinear weights do not reproduce them
    d6 = energy.derivative(case, T, 0, sign, inner)
    assert np.max(np.abs(d6 - (c[1] + 2 * c[2] * x[inner]))) > 1e-8


@pytest.mark.parametrize("dim", [2, 3])
def test_linear_field_moves_by_dt_u_grad_t_in_each_phase(dim):
    rng = np.random.Generator(np.random.PCG64(2 + dim))
    n = (12, 10, 9)
    case = energy_case(dim, n)
    x, y, z = cell_centres(case)
    gl, gv = rng.normal(size=3), rng.normal(size=3)
    if dim == 2:
        gl[2] = gv[2] = 0.0
    Tl = 300.0 + gl[0] * x + gl[1] * y + gl[2] * z
    Tv = 310.0 + gv[0] * x + gv[1] * y + gv[2] * z
    ul = [np.full(case.u_l[a].shape, s) for a, s in zip(range(dim), (0.7, -0.4, 0.0))]
    uv = [np.full(case.u_l[a].shape, s) for a, s in zip(range(dim), (-0.2, 0.0, 0.9))]
    dt = 0.1 * case.h
    got = energy.advect_energy(case, Tl, Tv, ul, uv, dt)
    col = case.ccol.ravel().astype(bool)
    vl = np.array([0.7, -0.4, 0.0][:dim])
    vv = np.array([-0.2, 0.0, 0.9][:dim])
    ex = np.where(col, Tl - dt * (vl @ gl[:dim]), Tv - dt * (vv @ gv[:dim]))
    # cells at least 2 away from every wall (the stencil is clamped there)
    far = np.ones(case.ncells, bool)
    for a, c in enumerate((x, y, z)[:dim]):
        far &= (c > 2 * case.h) & (c < case.n[a] * case.h - 2 * case.h)
    assert np.any(col[far]) and np.any(~col[far])
    assert np.max(np.abs(got[far] - ex[far])) < 1e-12


@pytest.mark.parametrize("u", [1.0, -1.0])
def test_step_moves_downstream_by_the_cfl_fraction(u):
    case = energy_case(2, (32, 4, 1), periodic=(False, True, False))
    x, _, _ = cell_centres(case)
    s = 16
    T = np.where(x > s * case.h, 1.0, 0.0)          # cells i >= s hold 1
    ul = [np.full(case.u_l[0].shape, u), np.zeros(case.u_l[1].shape)]
    cfl = 0.3
    dt = cfl * case.h / abs(u)
    got = energy.advect_energy(case, T, T, ul, ul, dt).reshape(4, 32)[0]
    want = T.reshape(4, 32)[0].copy()
    if u > 0:
        want[s] = 1.0 - cfl                           # the first high cell drops
    else:
        want[s - 1] = cfl                             # the last low cell rises
    assert np.max(np.abs(got - want)) < 1e-9


def _order(errs, ns):
    return np.log(errs[0] / errs[1]) / np.log(ns[1] / ns[0])


def test_derivative_converges_at_second_order_or_better():
    errs, ns = [], (64, 128)
    for n in ns:
        case = energy_case(2, (n, 4, 1), periodic=(True, True, False))
        x, _, _ = cell_centres(case)
        T = np.sin(2 * np.pi * x) + 0.3 * np.cos(4 * np.pi * x)
        dT = 2 * np.pi * np.cos(2 * np.pi * x) - 1.2 * np.pi * np.sin(4 * np.pi * x)
        d = energy.derivative(case, T, 0, 1, np.arange(case.ncells))
        errs.append(np.mean(np.abs(d - dT)))
    assert _order(errs, ns) > 1.9, errs


def test_shifting_a_periodic_field_shifts_the_result():
    rng = np.random.Generator(np.random.PCG64(7))
    case = energy_case(3, (10, 8, 6), periodic=(True, True, True), normal=(0.0, 0.0, 1.0), offset=2.0)
    assert case.ccol.max() == 0                       # one phase: shifts keep colours
    T = rough_field(case, rng)
    ul, uv = face_velocities(case, rng, 0.5)
    dt = 0.05
    base = energy.advect_energy(case, T, T, ul, uv, dt).reshape(6, 8, 10)
    sh = (2, 3, 5)                                    # cells along z, y, x
    Tr = np.roll(T.reshape(6, 8, 10), sh, axis=(0, 1, 2)).ravel()
    # roll the faces without their seam copy, then restore it
    faces = []
    for a, (u, shape) in enumerate(zip(uv, [(6, 8, 11), (6, 9, 10), (7, 8, 10)])):
        g = u.reshape(shape)
        ax = 2 - a
        core = np.roll(np.take(g, np.arange(g.shape[ax] - 1), axis=ax), sh, axis=(0, 1, 2))
        faces.append(np.concatenate([core, np.take(core, [0], axis=ax)], axis=ax).ravel())
    got = energy.advect_energy(case, Tr, Tr, faces, faces, dt).reshape(6, 8, 10)
    assert np.max(np.abs(got - np.roll(base, sh, axis=(0, 1, 2)))) < 1e-12


def test_mirroring_the_box_mirrors_the_step():
    rng = np.random.Generator(np.random.PCG64(8))
    case = energy_case(2, (20, 14, 1), normal=(0.0, 1.0, 0.0), offset=0.55)
    T = rough_field(case, rng).reshape(14, 20)
    ul, uv = face_velocities(case, rng, 0.5)
    dt = 0.1 * case.h
    base = energy.advect_energy(case, T.ravel(), T.ravel() + 1.0, ul, uv, dt).reshape(14, 20)
    # mirror x: cells reversed, x-faces reversed and negated, y-faces reversed
    mu = lambda f, a: (-f.reshape(14, 21)[:, ::-1] if a == 0 else f.reshape(15, 20)[:, ::-1]).ravel()
    got = energy.advect_energy(case, T[:, ::-1].ravel(), T[:, ::-1].ravel() + 1.0,
                               [mu(ul[0], 0), mu(ul[1], 1)], [mu(uv[0], 0), mu(uv[1], 1)], dt)
    assert np.max(np.abs(got.reshape(14, 20)[:, ::-1] - base)) < 1e-12


def test_zero_velocity_or_zero_dt_returns_t():
    rng = np.random.Generator(np.random.PCG64(9))
    case = energy_case(3, (7, 6, 5))
    Tl, Tv = rough_field(case, rng), rough_field(case, rng)
    col = case.ccol.ravel().astype(bool)
    z = [np.zeros(u.shape) for u in case.u_l]
    assert np.array_equal(energy.advect_energy(case, Tl, Tv, z, z, 0.3), np.where(col, Tl, Tv))
    ul, uv = face_velocities(case, rng, 1.0)
    assert np.array_equal(energy.advect_energy(case, Tl, Tv, ul, uv, 0.0), np.where(col, Tl, Tv))


def test_sampled_cells_equal_the_full_field():
    rng = np.random.Generator(np.random.PCG64(10))
    case = energy_case(3, (9, 8, 7), periodic=(True, False, True))
    Tl, Tv = smooth_field(case, rng), smooth_field(case, rng)
    ul, uv = face_velocities(case, rng, 1.0)
    full = energy.advect_energy(case, Tl, Tv, ul, uv, 0.01)
    cells = rng.choice(case.ncells, 50, replace=False)
    assert np.array_equal(energy.advect_energy(case, Tl, Tv, ul, uv, 0.01, cells=cells), full[cells])


@pytest.mark.parametrize("sign", [1, -1])
def test_stencils_stay_inside_walls(sign):
    """At the first and last cell of a wall axis the clamped stencil sees a
    flat continuation: a linear field's derivative there is at most half
    its slope; wrapping across the box (the periodic reading) would see the
    jump from one end of the ramp to the other."""
    b = 3.0
    for per in (False, True):
        case = energy_case(2, (16, 4, 1), periodic=(per, True, False))
        x, _, _ = cell_centres(case)
        T = b * x
        ends = np.nonzero((x < case.h) | (x > 1.0 - case.h))[0]
        d = energy.derivative(case, T, 0, sign, ends)
        if per:
            assert np.max(np.abs(d)) > 2.0 * b
        else:
            assert np.max(np.abs(d)) <= 0.5 * b * (1 + 1e-6)
