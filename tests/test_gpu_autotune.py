"""Autotuner: picks a schedule (nu1 = nu2, tail size, iteration-block
length) by timing solves; the tuned solves still meet the parity bar against
the oracle, for a context and for a batch."""
import sys

import numpy as np
import pytest

import ebit_inputs as ei
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _ebit():
    from paper_2402_13677_amd import ebit
    return ebit


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=float).ravel()
    b = np.asarray(b, dtype=float).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a)


def rhs_pair(ctx, dc):
    bh = torch.empty_like(dc.T0)
    ctx.heat_rhs(dc.T0, bh)
    m = torch.zeros_like(dc.T0)
    ctx.mass_flux(dc.T0, m)
    bp = torch.empty_like(dc.T0)
    ul = [u.clone() for u in dc.u_l]
    uv = [u.clone() for u in dc.u_v]
    ctx.project_rhs(ul, uv, m, bp)
    return bh, bp


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_context_autotune_then_parity(precision):
    ebit = _ebit()
    say(f"[gpu] autotune context ({precision})")
    c = ei.config(1, 48)
    opts = ebit.default_opts(rtol=1e-15, max_iters=400,
                             precision=ebit.MIXED if precision == "mixed" else ebit.FP64)
    ctx, dc = ebit.context_for(c, opts)
    ctx.build_coeffs(dc.markers, dc.vcol, dc.ccol, c.dt)
    bh, bp = rhs_pair(ctx, dc)
    chosen, ms = ctx.autotune(bh, bp)
    say("   chosen", chosen, f"{ms:.3f} ms")
    assert chosen["nu1"] == chosen["nu2"] and chosen["nu1"] in (1, 2, 3)
    assert chosen["tail_cells"] in (256, 1024, 4096, 16384) and chosen["check_every"] in (1, 2, 4)
    assert ms > 0 and np.isfinite(ms)
    ref = oracle.pipeline.run_step(c, c.T0, c.u_l, c.u_v)
    T = torch.zeros_like(dc.T0)
    ctx.heat_solve(dc.T0, T)
    m = torch.zeros_like(dc.T0)
    ctx.mass_flux(T, m)
    p = torch.zeros_like(dc.T0)
    ctx.project(dc.u_l, dc.u_v, m, p)
    for k, (g, o) in {"T": (T, ref["T"]), "mdot": (m, ref["mdot"]), "p": (p, ref["p"])}.items():
        e = rel(g.cpu().numpy(), o)
        say(f"   {k} {e:.1e}")
        assert e < 1e-12, (k, e)
    ctx.close()


def test_batch_autotune_then_parity():
    ebit = _ebit()
    say("[gpu] autotune batch")
    cases = ei.batch_cases(ncases=5, seed=4, sides=(16, 24, 32))
    opts = ebit.default_opts(rtol=1e-15, max_iters=400, precision=ebit.MIXED)
    ctxs, dcs = [], []
    for c in cases:
        ctx, dc = ebit.context_for(c, opts)
        ctxs.append(ctx)
        dcs.append(dc)
    b = ebit.Batch(ctxs)
    b.build_coeffs([d.markers for d in dcs], [d.vcol for d in dcs], [d.ccol for d in dcs], [c.dt for c in cases])
    pairs = [rhs_pair(ctx, dc) for ctx, dc in zip(ctxs, dcs)]
    chosen, ms = b.autotune([p[0] for p in pairs], [p[1] for p in pairs])
    say("   chosen", chosen, f"{ms:.3f} ms")
    T = [torch.zeros_like(d.T0) for d in dcs]
    b.heat_solve([d.T0 for d in dcs], T)
    for c, t in zip(cases, T):
        ref = oracle.pipeline.run_step(c, c.T0, c.u_l, c.u_v)
        e = rel(t.cpu().numpy(), ref["T"])
        assert e < 1e-12, (c.name, e)
    b.close()
    for x in ctxs:
        x.close()


def test_schedule_cache_context_and_batch(tmp_path):
    """ebit_autotune_cached: the first call times the candidates and appends
    the winner to the file; a second context (batch) of the same key takes
    it from the file without timing, gets the same schedule, and still
    meets the parity bar."""
    ebit = _ebit()
    path = tmp_path / "schedules.txt"
    c = ei.config(1, 48)
    opts = ebit.default_opts(rtol=1e-15, max_iters=400, precision=ebit.MIXED)
    say("[gpu] schedule cache: context")
    chosen = []
    for rep in range(2):
        ctx, dc = ebit.context_for(c, opts)
        ctx.build_coeffs(dc.markers, dc.vcol, dc.ccol, c.dt)
        bh, bp = rhs_pair(ctx, dc)
        ch, ms, hit = ctx.autotune_cached(path, bh, bp)
        assert hit == (rep == 1), (rep, hit)
        chosen.append((ch["nu1"], ch["tail_cells"], ch["check_every"]))
        if rep == 1:
            ref = oracle.pipeline.run_step(c, c.T0, c.u_l, c.u_v)
            T = torch.zeros_like(dc.T0)
            ctx.heat_solve(dc.T0, T)
            assert rel(T.cpu().numpy(), ref["T"]) < 1e-12
        ctx.close()
    assert chosen[0] == chosen[1]
    lines = [ln for ln in open(path) if ln.startswith("ebit-schedule")]
    assert len(lines) == 1
    say("[gpu] schedule cache: batch")
    cases = ei.batch_cases(ncases=4, seed=4, sides=(16, 24, 32))
    got = []
    for rep in range(2):
        ctxs, dcs = zip(*[ebit.context_for(x, opts) for x in cases])
        b = ebit.Batch(list(ctxs))
        b.build_coeffs([d.markers for d in dcs], [d.vcol for d in dcs], [d.ccol for d in dcs],
                       [x.dt for x in cases])
        pairs = [rhs_pair(cx, d) for cx, d in zip(ctxs, dcs)]
        ch, ms, hit = b.autotune_cached(path, [p[0] for p in pairs], [p[1] for p in pairs])
        assert hit == (rep == 1), (rep, hit)
        got.append((ch["nu1"], ch["tail_cells"], ch["check_every"]))
        b.close()
        for cx in ctxs:
            cx.close()
    assert got[0] == got[1]
    assert sum(1 for ln in open(path) if ln.startswith("ebit-schedule batch")) == 1
