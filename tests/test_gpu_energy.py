"""GPU parity of the energy advection step (ebit_advect_energy, Eq.
energy_advection) with the oracle (oracle/energy.py), through the C ABI.

Bar: element by element, |T*_gpu - T*_oracle| <= 8 ulp of max |T|.  T* =
T - dt sum_a u_a D_a.  The oracle forms each face value as a weighted mean
of values of size |T| (a few roundings), so its D_a carries an error of a
few ulp |T| / h; the kernel forms the face difference from one-sided
differences (the upwind cell plus half a weighted mean of differences,
both faces' quotients over one division), which is at least as accurate.
|u_a| dt <= CFL h turns a few ulp |T| / h into a few ulp |T| per axis (CFL
<= 0.5 in these cases); the final subtraction adds one more.  The choice
of the upwind side is taken on the same IEEE value of u_a on both sides.

Cases: 2D and 3D, walls and periodic axes, ragged sizes over several
blocks, smooth and rough (step plus cell-scale noise) per-phase fields,
face velocities of both signs with exact zeros; the 256 x 256 bubble in
full and the 256^3 film on sampled cells; dt = 0 returns T bit for bit;
argument errors.
"""
import zlib

import numpy as np
import pytest

import ebit_inputs as ei
from energy_util import cfl_dt, energy_case, face_velocities, rough_field, smooth_field
from oracle import energy
from parity_util import say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ULPS = 8


def _ebit():
    from paper_2402_13677_amd import ebit
    return ebit


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(np.asarray(x).ravel()), dtype=dtype).to("cuda")


def _bar(Tl, Tv):
    return ULPS * np.finfo(float).eps * max(float(np.max(np.abs(Tl))), float(np.max(np.abs(Tv))))


def _gpu(case, Tl, Tv, ul, uv, dt, eps=energy.WENO_EPS):
    ebit = _ebit()
    ctx, dc = ebit.context_for(case)
    out = torch.full((case.ncells,), float("nan"), dtype=torch.float64, device="cuda")
    ctx.advect_energy(dev(Tl), dev(Tv), [dev(u) for u in ul], [dev(u) for u in uv], dc.ccol, dt, out, eps=eps)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ctx, dc


CASES = [
    ("2d_walls_70x45_smooth", 2, (70, 45, 1), (False, False, False), "smooth"),
    ("2d_perx_64x33_rough", 2, (64, 33, 1), (True, False, False), "rough"),
    ("3d_walls_33x20x17_rough", 3, (33, 20, 17), (False, False, False), "rough"),
    ("3d_perxy_32x16x9_smooth", 3, (32, 16, 9), (True, True, False), "smooth"),
    ("3d_perz_19x23x32_rough", 3, (19, 23, 32), (False, False, True), "rough"),
    ("2d_tiny_4x5_rough", 2, (4, 5, 1), (True, False, False), "rough"),
]


@pytest.mark.parametrize("name,dim,n,per,kind", CASES, ids=[c[0] for c in CASES])
def test_energy_advection_parity(name, dim, n, per, kind):
    say(f"[gpu] energy advection {name}")
    case = energy_case(dim, n, periodic=per, name=name)
    rng = np.random.Generator(np.random.PCG64(zlib.crc32(name.encode())))
    gen = smooth_field if kind == "smooth" else rough_field
    Tl, Tv = gen(case, rng), gen(case, rng, base=380.0)
    ul, uv = face_velocities(case, rng, 0.02)
    dt = cfl_dt(case, ul, uv, 0.5)
    ref = energy.advect_energy(case, Tl, Tv, ul, uv, dt)
    got, _, _ = _gpu(case, Tl, Tv, ul, uv, dt)
    err = np.max(np.abs(got - ref))
    say(f"[gpu]   max |T* - oracle| = {err:.3e} (bar {_bar(Tl, Tv):.3e})")
    assert err <= _bar(Tl, Tv)
    # both phases and both signs were exercised
    col = case.ccol.ravel().astype(bool)
    assert np.any(col) and np.any(~col)


def test_eps_is_honoured():
    case = energy_case(3, (20, 16, 18), periodic=(False, True, False))
    rng = np.random.Generator(np.random.PCG64(31))
    Tl, Tv = rough_field(case, rng), rough_field(case, rng)
    ul, uv = face_velocities(case, rng, 0.02)
    dt = cfl_dt(case, ul, uv, 0.4)
    for eps in (1e-2, 1e-10):
        ref = energy.advect_energy(case, Tl, Tv, ul, uv, dt, eps=eps)
        got, _, _ = _gpu(case, Tl, Tv, ul, uv, dt, eps=eps)
        assert np.max(np.abs(got - ref)) <= _bar(Tl, Tv)


def test_zero_dt_returns_t_bit_for_bit():
    case = energy_case(3, (21, 14, 9))
    rng = np.random.Generator(np.random.PCG64(32))
    Tl, Tv = rough_field(case, rng), rough_field(case, rng)
    ul, uv = face_velocities(case, rng, 0.02)
    got, _, _ = _gpu(case, Tl, Tv, ul, uv, 0.0)
    col = case.ccol.ravel().astype(bool)
    assert np.array_equal(got, np.where(col, Tl, Tv))


def test_bubble2d_256_full():
    case = ei.config(1)
    rng = np.random.Generator(np.random.PCG64(33))
    Tl, Tv = smooth_field(case, rng), smooth_field(case, rng, base=380.0)
    ul, uv = face_velocities(case, rng, 0.05)
    dt = cfl_dt(case, ul, uv, 0.5)
    say("[gpu] energy advection bubble 256^2, full field")
    ref = energy.advect_energy(case, Tl, Tv, ul, uv, dt)
    got, _, _ = _gpu(case, Tl, Tv, ul, uv, dt)
    assert np.max(np.abs(got - ref)) <= _bar(Tl, Tv)


def test_film3d_256_sampled():
    """The 256^3 film (the benchmark's shape) in the launch the benchmark
    times, compared on 4000 sampled cells (those next to the interface and
    the walls among them)."""
    case = ei.film_3d(256)
    rng = np.random.Generator(np.random.PCG64(34))
    say("[gpu] energy advection film 256^3: fields")
    Tl, Tv = smooth_field(case, rng), smooth_field(case, rng, base=380.0)
    ul, uv = face_velocities(case, rng, 0.05)
    dt = cfl_dt(case, ul, uv, 0.5)
    say("[gpu] energy advection film 256^3: GPU")
    got, _, _ = _gpu(case, Tl, Tv, ul, uv, dt)
    col = case.ccol.ravel().astype(bool)
    iface = np.nonzero(col != np.roll(col, 1))[0]
    cells = np.unique(np.concatenate([rng.choice(case.ncells, 3000, replace=False),
                                      rng.choice(iface, min(800, iface.size), replace=False),
                                      np.arange(200), case.ncells - 1 - np.arange(200)]))
    ref = energy.advect_energy(case, Tl, Tv, ul, uv, dt, cells=cells)
    err = np.max(np.abs(got[cells] - ref))
    say(f"[gpu]   sampled max |T* - oracle| = {err:.3e}")
    assert err <= _bar(Tl, Tv)
    assert np.all(np.isfinite(got))


def test_errors():
    ebit = _ebit()
    case = energy_case(2, (16, 12, 1))
    ctx, dc = ebit.context_for(case)
    T = torch.zeros(case.ncells, dtype=torch.float64, device="cuda")
    out = torch.zeros_like(T)
    u = [torch.zeros(int(np.prod(ei.face_shape(2, case.n, a))), dtype=torch.float64, device="cuda")
         for a in range(2)]
    assert ctx.advect_energy(T, T, u, u, dc.ccol, -1.0, out, check=False) == ebit.EINVAL
    assert ctx.advect_energy(T, T, u, u, dc.ccol, float("nan"), out, check=False) == ebit.EINVAL
    assert ctx.advect_energy(T, T, u, u, dc.ccol, 0.1, out, eps=0.0, check=False) == ebit.EINVAL
    assert ctx.advect_energy(T, T, u, u, dc.ccol, 0.1, out, eps=1e-70, check=False) == ebit.EINVAL
    assert ctx.advect_energy(T, T, u, u, dc.ccol, 0.1, out, eps=float("inf"), check=False) == ebit.EINVAL
    assert ctx.advect_energy(T, T, u, u, dc.ccol, 0.1, T, check=False) == ebit.EINVAL
    assert ctx.advect_energy(T, T, u, u, dc.ccol, 0.1, out, check=False) == ebit.OK
