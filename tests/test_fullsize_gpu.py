"""Full-size parity of the run-based float32 path on the clumped 256^3 workload
(2^26 particles, half in 32 Gaussian clumps, sort every 4 steps) and the
batched workload (192^3 box with 4e7 charged, 8e6 dust and 1e6 tracer
particles plus 16 independent 64^3 boxes), in the launch configuration the
benchmark times.

Oracle checks that hold at this size: a sample of particles of every item,
advanced by the float64 oracle on its own (a particle's update reads only
the fields), compared per id; the grid-side and particle-side conservation
sums of every item (charge or dust mass equal to the particle count, J and F
grid sums equal to the particle-side sums).
"""

import sys

import numpy as np
import pytest

from tests import _cmp

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mods():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    from paper_2602_23434_amd import binding, driver, inputs
    binding.lib()
    return oracle, driver, inputs, binding


def _run(driver, B, wl, cfg, steps, every):
    from paper_2602_23434_amd import benchcfg as BC
    run = driver.Run(wl, **BC.run_kwargs(cfg))
    for s in range(steps):
        # the benchmark's sequence: a sorting step is one graph (sort, zero, step)
        fl = BC.STEP_FLAGS | (B.PL_SUMS if s == steps - 1 else 0) | (B.PL_SORT_FIRST if s % every == 0 else 0)
        run.step(flags=fl)
    assert run.sync() == B.PL_OK
    st = B.pl_part_stats(run.ctx)
    assert st[4] > 0 and st[5] == 0, st
    return run


def _check_sampled(oracle, wl, run, i, steps, nsample, seed, x_tol, u_tol):
    it = wl.items[i].particles
    box = wl.boxes[wl.items[i].box]
    sp = wl.species[wl.items[i].species]
    kind = oracle.KINDS[sp.kind]
    gx, gu, gid, _ = run.state(i)
    rng = np.random.default_rng(seed)
    sample = np.sort(rng.choice(it.n, min(nsample, it.n), replace=False))
    x = np.ascontiguousarray(it.x[:, sample])
    u = np.ascontiguousarray(it.u[:, sample])
    w = np.ascontiguousarray(it.w[sample])
    for _ in range(steps):
        oracle.step(3, box.n, oracle.TSC, (kind, sp.q, sp.m, sp.t_stop), x, u, w, box.fields, wl.dt)
    order = np.argsort(gid)
    gxs, gus = gx[:, order][:, sample], gu[:, order][:, sample]
    dx = np.abs(_cmp.min_image(gxs - x, box.n[0])).max()
    du = (np.sqrt(((gus - u) ** 2).sum(axis=0)) / np.maximum(np.sqrt((u * u).sum(axis=0)), 0.05)).max()
    say(f"  item {i} ({sp.kind}, {it.n} particles): sampled max |dx| {dx:.3e}, max |du|/max(|u|,sigma) {du:.3e}")
    assert dx <= x_tol and du <= u_tol, (i, dx, du)


def _check_sums(wl, sums, i, tol=1e-6):
    it = wl.items[i]
    sp = wl.species[it.species]
    if sp.kind == "tracer":
        return
    g, p = sums[i][:8], sums[i][8:]
    npart = it.particles.n
    expect = (sp.q if sp.kind == "lorentz" else sp.m) * npart
    assert abs(g[0] - expect) <= tol * expect and abs(p[0] - expect) <= tol * expect, (i, g[0], p[0], expect)
    chans = range(1, 7) if sp.kind == "lorentz" else range(4, 7)
    for ch in chans:
        assert abs(g[ch] - p[ch]) <= tol * max(abs(p[ch]), 1e-3 * npart * 0.05), (i, ch, g[ch], p[ch])


def test_clumped_256_fullsize(mods):
    oracle, driver, inputs, B = mods
    from paper_2602_23434_amd import benchcfg as BC
    say("[full] clumped 256^3, 2^26 particles (half in 32 clumps), 20 steps, sort every 4, f32 runs")
    wl = inputs.clumped_box()
    run = _run(driver, B, wl, BC.headline(), wl.steps, 4)
    _check_sampled(oracle, wl, run, 0, wl.steps, 2048, 21, 2e-5, 2e-5)
    _check_sums(wl, run.sums(), 0)
    run.close()


def test_batched_fullsize(mods):
    oracle, driver, inputs, B = mods
    from paper_2602_23434_amd import benchcfg as BC
    say("[full] batched: 192^3 box (charged, dust, tracers) + 16 boxes of 64^3, 20 steps, f32 runs")
    wl = inputs.batched()
    cfg = BC.batched_cfg()
    run = _run(driver, B, wl, cfg, wl.steps, cfg["sort_every"])
    sums = run.sums()
    for i in range(len(wl.items)):
        _check_sampled(oracle, wl, run, i, wl.steps, 1024 if i < 3 else 256, 31 + i, 2e-5, 2e-5)
        _check_sums(wl, sums, i)
    run.close()
