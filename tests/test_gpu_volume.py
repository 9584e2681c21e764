"""Liquid volume fraction (ebit_volume_fraction, 2D) through the C ABI
against the oracle (oracle/volume.py).

Bar: |GPU - oracle| <= 2 ulp of 1 per cell (fractions lie in [0, 1]).
Both sides form the same shoelace terms in the same order from the same
marker values (the kernel's file compiles with no fused multiply-adds), so
the results agree to the last bit or within a rounding of the final sum.

Cases: tilted lines of every orientation, discs of either colour, the
random circle and plane cases on ragged grids, the 256^2 bubble in full,
the 4096^2 bubble on every cell (cells without markers must be exactly
their colour; the interface cells are computed one by one by the oracle),
a grid with no interface; errors: a saddle cell (EGEOM, NaN there, every
other cell written), NULL arguments and a 3D context (EINVAL).
"""
import sys

import numpy as np
import pytest

import ebit_inputs as ei
from oracle import volume

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

BAR = 2 * np.finfo(float).eps


def _ebit():
    from paper_2402_13677_amd import ebit
    return ebit


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _case(n, ls, name="vf"):
    nn = (n[0], n[1], 1)
    h = 1.0 / max(n)
    vcol, ccol, mk = ei.colours_and_markers(2, nn, h, ls)
    zero = [np.zeros(ei.face_shape(2, nn, a)) for a in range(2)]
    return ei.Case(name, 2, nn, h, ei.Props(), 1e-4, [(0, 0.0)] * 4, [(1, 0.0)] * 4, mk, vcol, ccol,
                   np.zeros(ei.cell_shape(2, nn)), zero, [z.copy() for z in zero])


def _gpu(case):
    ebit = _ebit()
    ctx, dc = ebit.context_for(case)
    frac = torch.full((case.ncells,), -1.0, dtype=torch.float64, device="cuda")
    st = ctx.volume_fraction(dc.markers, dc.vcol, frac, check=False)
    out = frac.cpu().numpy().reshape(case.n[1], case.n[0])
    ctx.close()
    return st, out


CASES = [
    lambda: _case((24, 24), ei.Plane(np.array([0.8, 0.6, 0.0]), (0.52, 0.47, 0.0)), "line_a"),
    lambda: _case((31, 17), ei.Plane(np.array([-0.28, 0.96, 0.0]), (0.41, 0.25, 0.0)), "line_b"),
    lambda: _case((20, 33), ei.Plane(np.array([0.6, -0.8, 0.0]) / 1.0, (0.37, 0.61, 0.0)), "line_c"),
    lambda: _case((40, 40), ei.Plane(np.array([-0.95, -0.31, 0.0]) / np.hypot(0.95, 0.31), (0.58, 0.44, 0.0)),
                  "line_d"),
    lambda: _case((64, 64), ei.Ball((0.51, 0.47, 0.0), 0.23, 1.0, 2), "bubble_64"),
    lambda: _case((48, 37), ei.Ball((0.43, 0.36, 0.0), 0.17, -1.0, 2), "drop_48x37"),
    lambda: ei.random_case(2, 37, 3),
    lambda: ei.random_case(2, 45, 11, kind="plane"),
    lambda: ei.config(1),
]


@pytest.mark.parametrize("k", range(len(CASES)))
def test_volume_fraction_against_oracle(k):
    case = CASES[k]()
    say(f"[gpu] volume fraction {case.name} n={case.n}")
    ref = volume.volume_fraction(case)
    st, got = _gpu(case)
    assert st == _ebit().OK
    err = float(np.max(np.abs(got - ref)))
    say(f"[gpu]   max |GPU - oracle| = {err:.1e}; liquid area {got.sum() * case.h ** 2:.15f}")
    assert err <= BAR
    assert np.any((ref > 0) & (ref < 1))


def test_volume_fraction_4096_bubble():
    case = ei.config(1, n=4096)
    say("[gpu] volume fraction bubble 4096^2")
    st, got = _gpu(case)
    assert st == _ebit().OK
    n = case.n[0]
    vc = np.asarray(case.vcol).reshape(n + 1, n + 1)
    mx = np.asarray(case.markers[0]).reshape(n + 1, n)
    my = np.asarray(case.markers[1]).reshape(n, n + 1)
    cut = ~np.isnan(mx[:-1, :]) | ~np.isnan(mx[1:, :]) | ~np.isnan(my[:, :-1]) | ~np.isnan(my[:, 1:])
    assert np.array_equal(got[~cut], vc[:-1, :-1][~cut].astype(float))
    jj, ii = np.nonzero(cut)
    say(f"[gpu]   {jj.size} interface cells, each from the oracle")
    err = 0.0
    for j, i in zip(jj, ii):
        ref = volume.cell_fraction((vc[j, i], vc[j, i + 1], vc[j + 1, i + 1], vc[j + 1, i]),
                                   (mx[j, i], my[j, i + 1], mx[j + 1, i], my[j, i]))
        err = max(err, abs(got[j, i] - ref))
    assert err <= BAR


def test_volume_fraction_no_interface():
    case = _case((16, 12), ei.Plane(np.array([0.0, 1.0, 0.0]), (0.5, -0.5, 0.0)), "all_liquid")
    st, got = _gpu(case)
    assert st == _ebit().OK and np.all(got == 1.0)


def test_volume_fraction_saddle_and_errors():
    ebit = _ebit()
    n = 8
    case = _case((n, n), ei.Plane(np.array([0.0, 1.0, 0.0]), (0.5, -0.5, 0.0)), "saddle")
    vc = np.zeros((n + 1, n + 1), np.uint8)
    vc[3, 3] = vc[4, 4] = 1             # cell (3, 3) has liquid corners (3,3) and (4,4) only
    case.vcol[...] = vc.reshape(case.vcol.shape)
    mx = np.where(vc[:, :-1] != vc[:, 1:], 0.5, np.nan)
    my = np.where(vc[:-1, :] != vc[1:, :], 0.5, np.nan)
    case.markers[0][...] = mx.reshape(case.markers[0].shape)
    case.markers[1][...] = my.reshape(case.markers[1].shape)
    case.ccol[...] = 0
    st, got = _gpu(case)
    assert st == ebit.EGEOM
    assert np.isnan(got[3, 3])
    for j in range(n):
        for i in range(n):
            if (j, i) == (3, 3):
                continue
            ref = volume.cell_fraction((vc[j, i], vc[j, i + 1], vc[j + 1, i + 1], vc[j + 1, i]),
                                       (mx[j, i], my[j, i + 1], mx[j + 1, i], my[j, i]))
            assert abs(got[j, i] - ref) <= BAR, (j, i)
    # NULL arguments, a 3D context
    ctx, dc = ebit.context_for(case)
    frac = torch.zeros(case.ncells, dtype=torch.float64, device="cuda")
    assert ctx.volume_fraction(dc.markers, None, frac, check=False) == ebit.EINVAL
    assert ctx.volume_fraction(dc.markers, dc.vcol, None, check=False) == ebit.EINVAL
    assert ctx.lib.ebit_volume_fraction(ctx.h, ebit._P3(), ebit._ptr(dc.vcol, torch.uint8),
                                        ebit._ptr(frac, torch.float64)) == ebit.EINVAL
    ctx.close()
    c3 = ei.random_case(3, 8, 1)
    ctx, dc = ebit.context_for(c3)
    f3 = torch.zeros(c3.ncells, dtype=torch.float64, device="cuda")
    assert ctx.volume_fraction(dc.markers, dc.vcol, f3, check=False) == ebit.EINVAL
    ctx.close()
