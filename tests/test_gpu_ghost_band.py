"""Ghost velocities over the narrow band (ebit_ghost_band: Eq.
ghost_velocity with the band-extended mass flux, step 4 of the time
iteration) through the C ABI against the oracle (project.
ghost_velocities_band).

Bar: every face entry the oracle leaves alone is bit-identical to the input;
the others within 1e-12 |[1/rho]| max |mdot| plus 16 ulp of max |u| +
|[1/rho]| max |mdot|.  The ghost is u_real +- mdot_f [1/rho] n_f with the
same mdot on both sides; n_f is a facet normal (cut faces) or the mean of
two unit band normals, each the normalised sum of up to 3^d facet normals.
Each side builds its own facets, whose normals agree within 1e-12 (the
geometry parity bar; in 3D they come from an iterative eigen-solve), so n_f
agrees within about that, and the rest is rounding (the kernel may contract
a product into a fused multiply-add).

Cases: 2D and 3D, walls and periodic axes (the seam faces 0 and n both get
ghosts), balls of either colour, tilted planes, the film, a liquid slab
thinner than two cells (band cells whose block holds facets of both sides,
so their normals cancel to zero), ragged sizes; at full size the 256^2
bubble and the 256^3 film element by element; a grid with no interface
(nothing changes); argument errors.
"""
import sys

import numpy as np
import pytest

import ebit_inputs as ei
import oracle
from oracle import extend as oext
from oracle import project as oproj

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ULPS = 16


def _ebit():
    from paper_2402_13677_amd import ebit
    return ebit


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _slab_case():
    return ei.thin_slab_2d()


def _aniso3d():
    dim, n = 3, (70, 21, 19)
    h = 1.0 / 70
    ls = ei.Ball((0.47, 0.151, 0.137), 0.095, -1.0, dim)
    vcol, ccol, mk = ei.colours_and_markers(dim, n, h, ls)
    zero = [np.zeros(ei.face_shape(dim, n, a)) for a in range(dim)]
    return ei.Case("aniso3d", dim, n, h, ei.Props(), 2e-4, [(0, 0.0)] * 6, [(1, 0.0)] * 6, mk, vcol, ccol,
                   np.zeros(ei.cell_shape(dim, n)), zero, [z.copy() for z in zero])


def _check(case, seed, zero_normals=False):
    ebit = _ebit()
    geo = oracle.geometry.build(case)
    rng = np.random.default_rng(seed)
    mdot = rng.normal(0.0, 1.0, case.ncells)
    ul = [rng.normal(0.0, 1.0, ei.face_shape(case.dim, case.n, a)) for a in range(case.dim)]
    uv = [rng.normal(0.0, 1.0, ei.face_shape(case.dim, case.n, a)) for a in range(case.dim)]
    say(f"[gpu] band ghosts {case.name} n={case.n}: oracle")
    ref_l, ref_v = oproj.ghost_velocities_band(case, geo, mdot, ul, uv)
    if zero_normals:
        inb, nrm = oext.band(case, geo)
        assert np.any(inb & (np.abs(nrm).sum(axis=1) == 0)), "no band cell with a zero normal"
    say(f"[gpu] band ghosts {case.name}: GPU")
    ctx, dc = ebit.context_for(case)
    ctx.build_coeffs(dc.markers, dc.vcol, dc.ccol, case.dt)
    dl = [torch.from_numpy(np.ascontiguousarray(x).ravel()).to("cuda") for x in ul]
    dv = [torch.from_numpy(np.ascontiguousarray(x).ravel()).to("cuda") for x in uv]
    ctx.ghost_band(dl, dv, torch.from_numpy(mdot).to("cuda"))
    torch.cuda.synchronize()
    pr = case.props
    jc = abs(1.0 / pr.rho_l - 1.0 / pr.rho_v)
    scale = max(max(np.max(np.abs(x)) for x in ul), max(np.max(np.abs(x)) for x in uv)) + jc * np.max(np.abs(mdot))
    bar = 1e-12 * jc * np.max(np.abs(mdot)) + ULPS * np.finfo(float).eps * scale
    nghost = 0
    for a in range(case.dim):
        for name, dev, ref, inp in (("u_l", dl, ref_l, ul), ("u_v", dv, ref_v, uv)):
            got = dev[a].cpu().numpy().reshape(inp[a].shape)
            same = ref[a] == inp[a]
            assert np.array_equal(got[same], inp[a][same]), (case.name, name, a)
            err = float(np.max(np.abs(got - ref[a]))) if got.size else 0.0
            say(f"[gpu]   axis {a} {name}: {int((~same).sum())} ghosts, max err {err:.2e} (bar {bar:.2e})")
            assert err <= bar, (case.name, name, a, err, bar)
            nghost += int((~same).sum())
    assert nghost > 0
    ctx.close()


SMALL = [
    lambda: ei.config(0),
    lambda: ei.random_case(2, 37, 3),
    lambda: ei.random_case(2, 45, 11, kind="plane"),
    lambda: ei.random_case(3, 19, 5),
    lambda: ei.random_case(3, 16, 8, kind="plane"),
    lambda: ei.film_3d(32, name="film3d_32"),
    lambda: ei.config(1, n=96),
    _aniso3d,
]


@pytest.mark.parametrize("k", range(len(SMALL)))
def test_band_ghosts_small_against_oracle(k):
    _check(SMALL[k](), seed=100 + k)


def test_band_ghosts_thin_slab_zero_normals():
    _check(_slab_case(), seed=7, zero_normals=True)


@pytest.mark.parametrize("idx", [1, 4])
def test_band_ghosts_full_size(idx):
    _check(ei.config(idx), seed=200 + idx)


def test_band_ghosts_no_interface_changes_nothing():
    ebit = _ebit()
    case = ei.random_case(2, 24, 2)
    case.vcol[...] = 1
    case.ccol[...] = 1
    for m in case.markers:
        m[...] = np.nan
    ctx, dc = ebit.context_for(case)
    ctx.build_coeffs(dc.markers, dc.vcol, dc.ccol, case.dt)
    u0 = [torch.linspace(-1, 1, int(np.prod(ei.face_shape(2, case.n, a))), dtype=torch.float64, device="cuda")
          for a in range(2)]
    ul, uv = [x.clone() for x in u0], [-x for x in u0]
    m = torch.ones(case.ncells, dtype=torch.float64, device="cuda")
    ctx.ghost_band(ul, uv, m)
    torch.cuda.synchronize()
    assert all(torch.equal(x, y) for x, y in zip(ul, u0))
    assert all(torch.equal(x, -y) for x, y in zip(uv, u0))
    ctx.close()


def test_band_ghosts_argument_errors():
    ebit = _ebit()
    case = ei.random_case(2, 16, 1)
    ctx, dc = ebit.context_for(case)
    u = [torch.zeros(int(np.prod(ei.face_shape(2, case.n, a))), dtype=torch.float64, device="cuda")
         for a in range(2)]
    m = torch.zeros(case.ncells, dtype=torch.float64, device="cuda")
    assert ctx.ghost_band(u, u, m, check=False) == ebit.ESTATE      # before build_coeffs
    ctx.build_coeffs(dc.markers, dc.vcol, dc.ccol, case.dt)
    assert ctx.lib.ebit_ghost_band(ctx.h, ebit._P3(), ebit._P3(), None) == ebit.EINVAL
    assert ctx.lib.ebit_ghost_band(ctx.h, ebit._p3(u), ebit._p3(u), None) == ebit.EINVAL
    assert ctx.ghost_band(u, [u[0], None], m, check=False) == ebit.EINVAL
    assert ctx.ghost_band(u, u, m, check=False) == ebit.OK
    ctx.close()
