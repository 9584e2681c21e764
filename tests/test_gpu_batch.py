"""Batched solves (one launch per kernel over every case of a batch).

* A batch gives, case by case, exactly the results of the same calls on the
  single contexts (same kernels, same per-case reductions): compared bit for
  bit, over several steps so that the captured iteration blocks are replayed
  with the program's own eager work in between.
* Small uneven batches against the oracle (FP64 and mixed precision).
* The iteration-block length (check_every, graph replay) does not change
  any result.
* The 64-case uneven batch of sides 64..256 at full size: batch == single
  contexts bit for bit; sampled cases against the oracle.
* Invalid batches are rejected.
"""
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


class Fields:
    """Device fields of one case across steps."""

    def __init__(self, dc):
        self.T = dc.T0.clone()
        self.Tn = torch.zeros_like(dc.T0)
        self.m = torch.zeros_like(dc.T0)
        self.p = torch.zeros_like(dc.T0)
        self.u_l = [u.clone() for u in dc.u_l]
        self.u_v = [u.clone() for u in dc.u_v]

    def snapshot(self):
        return [x.clone() for x in [self.Tn, self.m, self.p] + self.u_l + self.u_v]


def run_single(cases, opts, steps):
    ebit = _ebit()
    out = []
    for c in cases:
        ctx, dc = ebit.context_for(c, opts)
        f = Fields(dc)
        snaps, its = [], []
        for _ in range(steps):
            ctx.build_coeffs(dc.markers, dc.vcol, dc.ccol, c.dt)
            sh = ctx.heat_solve(f.T, f.Tn)
            ctx.mass_flux(f.Tn, f.m)
            sp = ctx.project(f.u_l, f.u_v, f.m, f.p)
            f.T.copy_(f.Tn)
            snaps.append(f.snapshot())
            its.append((sh["iters"], sp["iters"]))
        ctx.close()
        out.append((snaps, its))
    return out


def run_batch(cases, opts, steps):
    ebit = _ebit()
    ctxs, dcs = [], []
    for c in cases:
        ctx, dc = ebit.context_for(c, opts)
        ctxs.append(ctx)
        dcs.append(dc)
    b = ebit.Batch(ctxs)
    fs = [Fields(dc) for dc in dcs]
    snaps = [[] for _ in cases]
    its = [[] for _ in cases]
    for _ in range(steps):
        b.build_coeffs([d.markers for d in dcs], [d.vcol for d in dcs], [d.ccol for d in dcs], [c.dt for c in cases])
        sh = b.heat_solve([f.T for f in fs], [f.Tn for f in fs])
        b.mass_flux([f.Tn for f in fs], [f.m for f in fs])
        sp = b.project([f.u_l for f in fs], [f.u_v for f in fs], [f.m for f in fs], [f.p for f in fs])
        for i, f in enumerate(fs):
            f.T.copy_(f.Tn)
            snaps[i].append(f.snapshot())
            its[i].append((sh[i]["iters"], sp[i]["iters"]))
    b.close()
    for c in ctxs:
        c.close()
    return list(zip(snaps, its))


def small_batch():
    cs = ei.batch_cases(ncases=6, seed=4, sides=(16, 24, 32, 40))
    cs.append(ei.random_case(2, 28, 3))
    return cs


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_equals_single_contexts(precision):
    ebit = _ebit()
    say(f"[gpu] batch == single contexts ({precision})")
    cases = small_batch()
    opts = ebit.default_opts(rtol=1e-12, precision=ebit.MIXED if precision == "mixed" else ebit.FP64)
    a = run_single(cases, opts, 3)
    b = run_batch(cases, opts, 3)
    for i, ((sa, ia), (sb, ib)) in enumerate(zip(a, b)):
        assert ia == ib, (i, ia, ib)
        for step, (xa, xb) in enumerate(zip(sa, sb)):
            for q, (u, v) in enumerate(zip(xa, xb)):
                assert torch.equal(u, v), (i, step, q)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_against_oracle(precision):
    ebit = _ebit()
    say(f"[gpu] batch vs oracle ({precision})")
    cases = small_batch()
    opts = ebit.default_opts(rtol=1e-15, max_iters=400,
                             precision=ebit.MIXED if precision == "mixed" else ebit.FP64)
    res = run_batch(cases, opts, 1)
    for c, (snaps, _) in zip(cases, res):
        ref = oracle.pipeline.run_step(c, c.T0, c.u_l, c.u_v)
        Tn, m, p = (x.cpu().numpy() for x in snaps[0][:3])
        errs = {"T": rel(Tn, ref["T"]), "mdot": rel(m, ref["mdot"]), "p": rel(p, ref["p"])}
        say(f"   {c.name} n={c.n[0]}", {k: f"{v:.1e}" for k, v in errs.items()})
        for k, v in errs.items():
            assert v < 1e-12, (c.name, k, v)


def test_iteration_block_length_does_not_change_results():
    ebit = _ebit()
    say("[gpu] check_every 1 vs 3 vs 5 (graph replays)")
    cases = small_batch()[:4]
    base = None
    for k in (1, 3, 5):
        opts = ebit.default_opts(rtol=1e-12, precision=ebit.MIXED, check_every=k)
        r = run_batch(cases, opts, 3)
        if base is None:
            base = r
            continue
        for (sa, ia), (sb, ib) in zip(base, r):
            assert ia == ib
            for xa, xb in zip(sa, sb):
                for u, v in zip(xa, xb):
                    assert torch.equal(u, v)


def test_invalid_batches_rejected():
    ebit = _ebit()
    say("[gpu] batch einval")
    c2 = ei.random_case(2, 16, 1)
    c3 = ei.random_case(3, 8, 1)
    a, _ = ebit.context_for(c2)
    b, _ = ebit.context_for(c3)
    with pytest.raises(ebit.EbitError) as e:
        ebit.Batch([a, b])          # different dims
    assert e.value.status == ebit.EINVAL
    with pytest.raises(ebit.EbitError) as e:
        ebit.Batch([a, a])          # the same context twice
    assert e.value.status == ebit.EINVAL
    m, _ = ebit.context_for(c2, ebit.default_opts(precision=ebit.MIXED))
    with pytest.raises(ebit.EbitError) as e:
        ebit.Batch([a, m])          # different solver options
    assert e.value.status == ebit.EINVAL
    for x in (a, b, m):
        x.close()


def test_c4_uneven_batch_full_size():
    """64 cases, sides 64..256, mixed precision, rtol 1e-9: one step."""
    ebit = _ebit()
    say("[gpu] C4 64-case batch, full size")
    cases = ei.config(3)
    opts = ebit.default_opts(rtol=1e-9, precision=ebit.MIXED)
    b = run_batch(cases, opts, 1)
    sample = [0, 1, 2, 3]
    a = run_single([cases[i] for i in range(len(cases))], opts, 1)
    for i, ((sa, ia), (sb, ib)) in enumerate(zip(a, b)):
        assert ia == ib, (i, ia, ib)
        for xa, xb in zip(sa[0], sb[0]):
            assert torch.equal(xa, xb), i
    # sampled cases against the oracle's own operators: residual of T and p
    for i in sample:
        c = cases[i]
        geo = oracle.geometry.build(c)
        opH = oracle.heat.operator(c, geo)
        bH = oracle.heat.rhs(c, geo, c.T0)
        Tn = b[i][0][0][0].cpu().numpy().ravel()
        rr = np.linalg.norm(bH - opH.matvec(Tn)) / np.linalg.norm(bH)
        say(f"   case {i} n={c.n[0]}: heat residual under the oracle operator {rr:.1e}")
        assert rr < 2e-9
        mo, _ = oracle.flux.mass_flux(c, geo, Tn.reshape(c.T0.shape))
        m = b[i][0][0][1].cpu().numpy().ravel()
        assert rel(m, mo) < 1e-12


def test_c4_batch_every_schedule_many_steps():
    """The 64-case batch over every candidate schedule (nu x tail x block
    length), 8 steps each: every solve converges (a block of the first fine
    sweep that read the case's control word while block 0 was ending the
    previous iteration once took the other branch, so its waves missed each
    other's barriers; such a case ended in NaN now and then)."""
    import itertools
    ebit = _ebit()
    say("[gpu] C4 batch, every schedule, 8 steps")
    cases = ei.config(3)
    for nu, tail, k in itertools.product((1, 2, 3), (256, 1024, 4096, 16384), (1, 2, 4)):
        opts = ebit.default_opts(rtol=1e-9, precision=ebit.MIXED, nu1=nu, nu2=nu, tail_cells=tail, check_every=k)
        ctxs, dcs = [], []
        for c in cases:
            ctx, dc = ebit.context_for(c, opts)
            ctxs.append(ctx)
            dcs.append(dc)
        fs = [Fields(dc) for dc in dcs]
        b = ebit.Batch(ctxs)
        for s in range(8):
            b.build_coeffs([d.markers for d in dcs], [d.vcol for d in dcs], [d.ccol for d in dcs],
                           [c.dt for c in cases])
            sh = b.heat_solve([f.T for f in fs], [f.Tn for f in fs])
            b.mass_flux([f.Tn for f in fs], [f.m for f in fs])
            sp = b.project([f.u_l for f in fs], [f.u_v for f in fs], [f.m for f in fs], [f.p for f in fs])
            assert all(x["status"] == 0 for x in sh + sp), (nu, tail, k, s)
            for f in fs:
                f.T.copy_(f.Tn)
        b.close()
        for c in ctxs:
            c.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_3d_equals_single_contexts(precision):
    """An uneven 3D batch (walls and a periodic film; sides 12 to 21): the
    3D work lists (tiles x z-chunks per case) give each case exactly the
    single-context results."""
    ebit = _ebit()
    say(f"[gpu] 3D batch == single contexts ({precision})")
    cases = [ei.random_case(3, 12, 21), ei.random_case(3, 17, 22, kind="plane"), ei.film_3d(16, name="film16"),
             ei.random_case(3, 21, 23)]
    opts = ebit.default_opts(rtol=1e-12, precision=ebit.MIXED if precision == "mixed" else ebit.FP64)
    a = run_single(cases, opts, 2)
    b = run_batch(cases, opts, 2)
    for i, ((sa, ia), (sb, ib)) in enumerate(zip(a, b)):
        assert ia == ib, (i, ia, ib)
        for step, (xa, xb) in enumerate(zip(sa, sb)):
            for q, (u, v) in enumerate(zip(xa, xb)):
                assert torch.equal(u, v), (i, step, q)


def test_batch_null_argument_launches_nothing():
    """A NULL field for a later case is refused with EBIT_EINVAL before any
    case's kernels are queued: the earlier cases' outputs stay untouched."""
    import ctypes
    ebit = _ebit()
    say("[gpu] batch NULL argument of case 1 launches nothing")
    cases = [ei.random_case(2, 20, 3), ei.random_case(2, 24, 4)]
    ctxs, dcs = zip(*[ebit.context_for(c) for c in cases])
    b = ebit.Batch(list(ctxs))
    b.build_coeffs([d.markers for d in dcs], [d.vcol for d in dcs], [d.ccol for d in dcs],
                   [c.dt for c in cases])
    T = [torch.zeros_like(d.T0) for d in dcs]
    b.heat_solve([d.T0 for d in dcs], T)
    m0 = torch.full_like(T[0], 7.0)
    arr_T = (ctypes.c_void_p * 2)(T[0].data_ptr(), T[1].data_ptr())
    arr_m = (ctypes.c_void_p * 2)(m0.data_ptr(), None)
    st = b.lib.ebit_batch_mass_flux(b.h, arr_T, arr_m, None)
    torch.cuda.synchronize()
    assert st == ebit.EINVAL
    assert torch.all(m0 == 7.0)
    p0 = torch.full_like(T[0], 5.0)
    u0 = [u.clone() for u in dcs[0].u_l]
    arr_p = (ctypes.c_void_p * 2)(p0.data_ptr(), None)
    arr_md = (ctypes.c_void_p * 2)(m0.data_ptr(), m0.data_ptr())
    st = b.lib.ebit_batch_project(b.h, ebit._ptrs([d.u_l for d in dcs], per=3),
                                  ebit._ptrs([d.u_v for d in dcs], per=3), arr_md, arr_p, 0, None)
    torch.cuda.synchronize()
    assert st == ebit.EINVAL
    assert torch.all(p0 == 5.0)
    for a in range(2):
        assert torch.equal(u0[a], dcs[0].u_l[a])
    b.close()
    for x in ctxs:
        x.close()
