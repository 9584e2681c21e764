"""Determinism: the same steps on two fresh contexts give the same bits.

Every reduction runs in a fixed order and no sweep reads a buffer that the
same launch writes (the launches of a level alternate between its two
iterate buffers), so the results cannot depend on the order in which the
work-groups run.  Checked over two steps (graph capture, then replay) for a
2D bubble in FP64 and mixed precision, a 2D grid of odd size, and a small
3D film that is periodic along x and z.

In 2D the strided p-update with 64-bit cell offsets (used from 2^30 cells
on) gives the same bits as the 32-bit one: forced on with
EBIT_WIDE_OFFSETS=1, heat and pressure, FP64 and mixed.  (In 3D the switch
replaces the LDS-staged p-update, whose p.q partial sums group the cells
differently; the parity tests run that form against the oracle.)
"""
import os
import sys

import pytest

import ebit_inputs as ei

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run(case, opts, steps):
    from paper_2402_13677_amd import ebit
    ctx, dc = ebit.context_for(case, opts)
    T = dc.T0.clone()
    Tn = torch.zeros_like(T)
    m = torch.zeros_like(T)
    p = torch.zeros_like(T)
    u_l = [u.clone() for u in dc.u_l]
    u_v = [u.clone() for u in dc.u_v]
    its = []
    for _ in range(steps):
        ctx.build_coeffs(dc.markers, dc.vcol, dc.ccol, case.dt)
        sh = ctx.heat_solve(T, Tn)
        ctx.mass_flux(Tn, m)
        sp = ctx.project(u_l, u_v, m, p)
        T.copy_(Tn)
        its.append((sh["iters"], sp["iters"]))
    torch.cuda.synchronize()
    out = [x.cpu() for x in [Tn, m, p] + u_l + u_v]
    ctx.close()
    return out, its


CASES = [
    ("bubble2d_96_fp64", 1, 96, "fp64"),
    ("bubble2d_96_mixed", 1, 96, "mixed"),
    ("bubble2d_45_mixed", 1, 45, "mixed"),
    ("film3d_32_mixed", 4, 32, "mixed"),
]


@pytest.mark.parametrize("name,idx,n,prec", CASES, ids=[c[0] for c in CASES])
def test_repeat_is_bit_identical(name, idx, n, prec):
    from paper_2402_13677_amd import ebit
    say(f"[gpu] determinism {name}")
    case = ei.config(idx, n)
    opts = ebit.default_opts(rtol=1e-10, precision=ebit.MIXED if prec == "mixed" else ebit.FP64)
    a, ia = run(case, opts, 2)
    b, ib = run(case, opts, 2)
    assert ia == ib, (ia, ib)
    for k, (x, y) in enumerate(zip(a, b)):
        assert torch.equal(x, y), (name, k)


WIDE = [
    ("bubble2d_96_mixed", 1, 96, "mixed"),
    ("bubble2d_45_fp64", 1, 45, "fp64"),
]


@pytest.mark.parametrize("name,idx,n,prec", WIDE, ids=[c[0] for c in WIDE])
def test_wide_offsets_are_bit_identical(name, idx, n, prec):
    from paper_2402_13677_amd import ebit
    say(f"[gpu] 64-bit offsets {name}")
    case = ei.config(idx, n)
    opts = ebit.default_opts(rtol=1e-10, precision=ebit.MIXED if prec == "mixed" else ebit.FP64)
    a, ia = run(case, opts, 2)
    os.environ["EBIT_WIDE_OFFSETS"] = "1"
    try:
        b, ib = run(case, opts, 2)
    finally:
        del os.environ["EBIT_WIDE_OFFSETS"]
    assert ia == ib, (ia, ib)
    for k, (x, y) in enumerate(zip(a, b)):
        assert torch.equal(x, y), (name, k)
