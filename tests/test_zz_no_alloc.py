"""The geometry pass without allocation (ebit_cut_fractions_noalloc) against
the same pass of ebit_build_coeffs (read back with ebit_get_geometry), through
the C ABI: bit-identical theta and flags on two calls in a row, the second on
a smaller grid (the shared scratch array keeps the first call's contents);
a grid above the maximum is refused with EBIT_EINVAL before any launch;
inconsistent markers give EBIT_EGEOM."""
import numpy as np
import pytest

import ebit_inputs as ei
from parity_util import say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _ebit():
    from paper_2402_13677_amd import ebit
    return ebit


def _context_geometry(case):
    ebit = _ebit()
    ctx, dc = ebit.context_for(case)
    ctx.build_coeffs(dc.markers, dc.vcol, dc.ccol, case.dt)
    th = [torch.empty(ei.face_shape(case.dim, case.n, a), dtype=torch.float64, device="cuda")
          for a in range(case.dim)]
    fl = torch.empty(case.ncells, dtype=torch.uint8, device="cuda")
    ctx.get_geometry(th, fl, None)
    torch.cuda.synchronize()
    ctx.close()
    return [t.cpu().numpy() for t in th], fl.cpu().numpy(), dc


def _noalloc_geometry(case, dc):
    ebit = _ebit()
    th = [torch.full(ei.face_shape(case.dim, case.n, a), 3.0, dtype=torch.float64, device="cuda")
          for a in range(case.dim)]
    fl = torch.full((case.ncells,), 0xAA, dtype=torch.uint8, device="cuda")
    st = ebit.cut_fractions_noalloc(dc.grid, dc.markers, dc.vcol, dc.ccol, th, fl)
    torch.cuda.synchronize()
    return st, [t.cpu().numpy() for t in th], fl.cpu().numpy()


def _same(a, b):
    """Bit-identical float arrays (NaN where the other has NaN)."""
    return np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_noalloc_equals_build_coeffs_on_two_calls():
    say("[gpu] no-alloc geometry: 64^3 sphere then a 100 x 90 circle")
    n2 = (100, 90, 1)
    vcol, ccol, mk = ei.colours_and_markers(2, n2, 1.0 / 100, ei.Ball((0.47, 0.43, 0.0), 0.21, 1.0, 2))
    small = ei.Case("ball2d_100x90", 2, n2, 1.0 / 100, ei.Props(), 1e-4, [(0, 0.0)] * 4, [(1, 0.0)] * 4,
                    mk, vcol, ccol, np.zeros(ei.cell_shape(2, n2)), [], [])
    cases = [ei.bubble(3, 64, 0.2, 1.0, 0.05, 100.0, 0.2, name="ball3d_64"), small]
    assert cases[0].ncells == _ebit().NOALLOC_MAX_CELLS and cases[1].ncells < cases[0].ncells
    for case in cases:
        th_ref, fl_ref, dc = _context_geometry(case)
        st, th, fl = _noalloc_geometry(case, dc)
        say(f"   {case.name}: status {st}, {int(np.count_nonzero(fl_ref & 0x80))} interface cells")
        assert st == 0
        assert np.array_equal(fl, fl_ref)
        for a in range(case.dim):
            assert _same(th[a], th_ref[a]), a


def test_noalloc_refuses_a_grid_above_the_maximum():
    ebit = _ebit()
    say("[gpu] no-alloc geometry: grid above the maximum")
    case = ei.random_case(2, 520, 1)          # 270,400 cells > 2^18
    dc = ebit.DeviceCase(case)
    th = [torch.full(ei.face_shape(2, case.n, a), 3.0, dtype=torch.float64, device="cuda") for a in range(2)]
    fl = torch.full((case.ncells,), 7, dtype=torch.uint8, device="cuda")
    st = ebit.cut_fractions_noalloc(dc.grid, dc.markers, dc.vcol, dc.ccol, th, fl)
    torch.cuda.synchronize()
    assert st == ebit.EINVAL
    assert torch.all(fl == 7) and all(torch.all(t == 3.0) for t in th)


def test_noalloc_inconsistent_markers_give_egeom():
    ebit = _ebit()
    say("[gpu] no-alloc geometry: inconsistent markers")
    case = ei.random_case(2, 32, 2)
    mk = [m.copy() for m in case.markers]
    j, i = np.argwhere(np.isnan(mk[0][0]))[0]
    mk[0][0, j, i] = 0.5                       # a marker on an edge whose ends share a colour
    case.markers = mk
    dc = ebit.DeviceCase(case)
    th = [torch.empty(ei.face_shape(2, case.n, a), dtype=torch.float64, device="cuda") for a in range(2)]
    fl = torch.empty(case.ncells, dtype=torch.uint8, device="cuda")
    assert ebit.cut_fractions_noalloc(dc.grid, dc.markers, dc.vcol, dc.ccol, th, fl) == ebit.EGEOM
    # the next call clears the status word: a consistent grid succeeds
    ok = ei.random_case(2, 32, 2)
    dc2 = ebit.DeviceCase(ok)
    assert ebit.cut_fractions_noalloc(dc2.grid, dc2.markers, dc2.vcol, dc2.ccol, th, fl) == 0
