"""The Lagrangian-particle extras on the GPU through the C ABI, against the
float64 oracle: the spectral update (Sec. 2, Eqs. cr_N to cr_chi and
rad_losses), deletion at open boundaries with the holes-and-fillers
compaction (Sec. 3.2), and injection.

Tolerances.  Spectra, float64 form: 1e-13 relative per value after three
steps (the oracle and the kernel evaluate the same closed form; they differ
by the rounding of exp, expm1 and one reciprocal, a few ulp per step).
Float32 form: the particle position carries the float32 offset's rounding
(up to 2^-25 ~ 3e-8 cells), which moves the sampled a and c_r by that times
their relative gradient (about 1.6 per cell for these 16^3 fields, modes up
to |m| = 4); energies and chi move by that times the step's exponents
(|a d tau| + c_r eps d tau, up to about 2.5 here): 3e-8 * 1.6 * 2.5 ~ 1.2e-7,
so 2e-7 relative (measured 2.7e-8).  The compaction is index work:
bit-exact.
"""

import sys

import numpy as np
import pytest

from tests import _cmp

pytestmark = pytest.mark.gpu

CR, U_RAD, UB = 2e-4, 0.1, 0.5


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


def _spectra_wl(inputs, n=16, ppc=4, nb=128, steps=3, shape="tsc"):
    wl = inputs.spectra_box(n=n, ppc=ppc, nb=nb, steps=steps, divu_rms=2.0, dt=0.5)
    wl.shape = shape
    return wl


def _oracle_spectra(oracle, wl, x, steps):
    eng = np.ascontiguousarray(np.broadcast_to(wl.notes["eng0"], (x.shape[1], len(wl.notes["eng0"]))))
    chi = np.ascontiguousarray(np.broadcast_to(wl.notes["chi0"], eng.shape))
    box = wl.boxes[0]
    shape = oracle.SHAPES[wl.shape]
    for _ in range(steps):
        oracle.spectra_step(box.ndim, box.n, shape, x, box.fields, box.fields["divu"], eng, chi, wl.dt,
                            cr=CR, u_rad=U_RAD, ub=UB)
    return eng, chi


@pytest.mark.parametrize("prec,shape,n", [("f64", "tsc", 16), ("f32", "tsc", 16), ("f64", "cic", 16),
                                          ("f64", "tsc", (20, 12, 16)), ("f32", "tsc", (20, 12, 16))])
def test_spectra_vs_oracle(mods, prec, shape, n):
    oracle, driver, inputs, B = mods
    wl = _spectra_wl(inputs, n=n, shape=shape)
    npart = wl.items[0].particles.n
    say(f"[lp] spectra {prec} {shape}: {wl.boxes[0].n}, {npart} particles x 128 points, 3 steps")
    p = B.PL_F64 if prec == "f64" else B.PL_F32_OFFSET
    run = driver.Run(wl, prec=p, algo=B.PL_ALGO_PLAIN, spectra=True)
    for _ in range(wl.steps):
        run.spectra(cr=CR, u_rad=U_RAD, ub=UB)
    assert run.sync() == B.PL_OK
    ge, gc = run.spectra_state(0)
    oe, oc = _oracle_spectra(oracle, wl, wl.items[0].particles.x.copy(), wl.steps)
    tol = 1e-13 if p == B.PL_F64 else 2e-7
    re = np.abs(ge - oe) / oe
    rc = np.abs(gc - oc) / oc
    say(f"  max rel error: eng {re.max():.2e}, chi {rc.max():.2e}; "
        f"eng moved by up to {np.abs(oe / wl.notes['eng0'] - 1).max():.2e}")
    assert re.max() <= tol and rc.max() <= tol
    # the losses and the adiabatic term both acted
    assert np.abs(oe / wl.notes["eng0"] - 1).max() > 0.05
    run.close()


@pytest.mark.parametrize("algo", ["tiled", "runs"])
def test_spectra_move_with_sort_and_push(mods, algo):
    """The paper's particle step, two RK stages then the spectral update
    (Table 1 order), with a sort every 2 steps: the spectral rows travel
    with their particles through the sort (in run order through the run
    table's permutation composed with the tile+cell one), so per id they
    match the oracle's."""
    oracle, driver, inputs, B = mods
    wl = _spectra_wl(inputs, steps=4)
    wl.dt = 0.4
    say(f"[lp] tracers + spectra, 16^3, float64 {algo} kernel, sort every 2 steps")
    if algo == "tiled":
        kw = dict(algo=B.PL_ALGO_TILED)
    else:
        kw = dict(algo=B.PL_ALGO_RUNS, key_mode=B.PL_KEY_TILE_RUN, block=512)
    run = driver.Run(wl, prec=B.PL_F64, tile=(4, 4, 4), spectra=True, **kw)
    for s in range(wl.steps):
        if s % 2 == 0:
            run.sort()
        run.step(flags=0)
        run.spectra(cr=CR, u_rad=U_RAD, ub=UB)
    assert run.sync() == B.PL_OK
    gx, gu, gid, _ = run.state(0)
    ge, gc = run.spectra_state(0)
    assert not np.array_equal(gid, np.arange(len(gid)))          # the sort reordered them
    box = wl.boxes[0]
    x = wl.items[0].particles.x.copy()
    u = wl.items[0].particles.u.copy()
    eng = np.ascontiguousarray(np.broadcast_to(wl.notes["eng0"], (x.shape[1], 128)))
    chi = np.ascontiguousarray(np.broadcast_to(wl.notes["chi0"], eng.shape))
    for _ in range(wl.steps):
        oracle.step(3, box.n, oracle.TSC, (oracle.TRACER, 0.0, 1.0, 0.0), x, u, None, box.fields, wl.dt)
        oracle.spectra_step(3, box.n, oracle.TSC, x, box.fields, box.fields["divu"], eng, chi, wl.dt,
                            cr=CR, u_rad=U_RAD, ub=UB)
    ex, _ = _cmp.state_errors(gx, gu, gid, x, u, box.n, 3)
    assert ex <= 1e-11
    order = np.argsort(gid)
    re = (np.abs(ge[order] - eng) / eng).max()
    rc = (np.abs(gc[order] - chi) / chi).max()
    say(f"  position error {ex:.2e} cells; spectra max rel error eng {re:.2e} chi {rc:.2e}")
    assert re <= 1e-12 and rc <= 1e-12
    run.close()


@pytest.mark.parametrize("n", [16, (20, 12, 16)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_boundary_compaction_exact(mods, prec, n):
    """Particles placed over the whole box (16^3, or 20x12x16 so that a
    swapped dimension shows), sorted by tile, one spectral step, then x and z
    opened with two ghost layers: the GPU deletes and compacts
    exactly as the oracle's holes-and-fillers algorithm does on the oracle's
    own sorted state (stable tile sort, spectra at the same positions), every
    array including the spectral rows moving with its particle; the item is
    unsorted afterwards."""
    oracle, driver, inputs, B = mods
    tile = (4, 4, 4)
    wl = _spectra_wl(inputs, n=n, ppc=4, nb=16, steps=1)
    box = wl.boxes[0]
    p = B.PL_F64 if prec == "f64" else B.PL_F32_OFFSET
    n0 = wl.items[0].particles.n
    say(f"[lp] boundary {prec}: {box.n} open in x and z, ghost 2, {n0} particles")
    run = driver.Run(wl, prec=p, algo=B.PL_ALGO_TILED, tile=tile, spectra=True)
    run.sort()
    run.spectra(cr=CR, u_rad=U_RAD, ub=UB)            # rows now differ from particle to particle
    assert run.sync() == B.PL_OK
    removed = run.boundary((1, 0, 1), 2)

    # the oracle's state before the boundary call: stable tile sort of the
    # seeded positions, one spectral step there
    x_in = wl.items[0].particles.x
    if p == B.PL_F64:
        cells = oracle.cells_of_positions(3, box.n, x_in)
    else:
        cells, offs = oracle.split_positions(3, box.n, x_in)
    keys = np.array([oracle.tile_key(3, box.n, tile, 0, *cells[:, q]) for q in range(n0)], dtype=np.uint32)
    perm = oracle.stable_sort_perm(keys)
    xo = np.ascontiguousarray(x_in[:, perm])
    eng, chi = _oracle_spectra(oracle, wl, xo, 1)
    if p == B.PL_F64:
        flag = oracle.outside(3, box.n, (1, 0, 1), 2, xo)
        cols = [perm.astype(np.uint64)] + [np.ascontiguousarray(xo[a]) for a in range(3)]
    else:
        # the float32 form's cell (an offset that rounds to +1/2 moves on) decides
        cp, op = cells[:, perm], offs[:, perm]
        flag = oracle.outside(3, box.n, (1, 0, 1), 2, cp + 0.5 + op.astype(np.float64))
        packed = (cp[0] | (cp[1] << 10) | (cp[2] << 20)).astype(np.uint32)
        cols = [perm.astype(np.uint64), packed] + [np.ascontiguousarray(op[a]) for a in range(3)]
    cols += [eng, chi]
    keep, holes, fills = oracle.compact(flag, cols)
    say(f"  removed {removed[0]} of {n0}; {len(holes)} holes filled")
    assert removed == [n0 - keep] and run.items[0].p.n == keep and 0 < len(holes) < keep

    after = run.raw(0)
    assert np.array_equal(after["id"][:keep].astype(np.uint64), cols[0][:keep])
    k = 1
    if p == B.PL_F32_OFFSET:
        assert np.array_equal(after["cell"][:keep].view(np.uint32), cols[1][:keep])
        k = 2
    for a in range(3):
        assert np.array_equal(after["x"][a][:keep], cols[k + a][:keep]), a
    ge, gc = run.spectra_state(0)
    tol = 1e-13 if p == B.PL_F64 else 2e-7
    assert (np.abs(ge - cols[-2][:keep]) / cols[-2][:keep]).max() <= tol
    assert (np.abs(gc - cols[-1][:keep]) / cols[-1][:keep]).max() <= tol
    # the order changed: tiled steps wait for a sort
    run.step(flags=0)
    assert run.sync() == B.PL_ENOTSORTED
    run.sort()
    run.step(flags=0)
    assert run.sync() == B.PL_OK
    run.close()


def test_open_box_outflow_and_injection(mods):
    """Tracers in a uniform flow through a box open in x (plain float64
    kernel): every step pushes, deletes what left and injects new particles
    at the inflow face.  The surviving ids equal the oracle's run of the same
    pipeline, and positions match per id."""
    oracle, driver, inputs, B = mods
    n = (32, 8, 8)
    g = 2
    rng = np.random.default_rng(9)
    npart = 3000
    x = np.zeros((3, npart))
    x[0] = g + rng.random(npart) * (n[0] - 2 * g)
    x[1] = rng.random(npart) * n[1]
    x[2] = rng.random(npart) * n[2]
    f = inputs.uniform_fields(n, vg=(0.45, 0.05, 0.0))
    box = inputs.Box(3, n, {"vg": f["vg"]})
    wl = inputs.Workload(name="open box", boxes=[box], species=[inputs.Species("tracer")],
                         items=[inputs.Item(0, 0, inputs.make_particles(x, np.zeros((3, npart))))],
                         dt=1.0, steps=12)
    say("[lp] open box: uniform flow, push + delete + inject for 12 steps, f64 plain")
    run = driver.Run(wl, prec=B.PL_F64, algo=B.PL_ALGO_PLAIN, capacity=2 * npart)
    ox, oids = x.copy(), np.arange(npart, dtype=np.uint64)
    next_id = npart
    for s in range(wl.steps):
        run.step(flags=0)
        removed = run.boundary((1, 0, 0), g)
        xs, us = np.ascontiguousarray(ox), np.zeros_like(ox)
        oracle.step(3, n, oracle.TSC, (oracle.TRACER, 0.0, 1.0, 0.0), xs, us, None, box.fields, wl.dt)
        flag = oracle.outside(3, n, (1, 0, 0), g, xs)
        cols = [np.ascontiguousarray(xs[a]) for a in range(3)] + [oids.copy()]
        keep, _, _ = oracle.compact(flag, cols)
        assert removed == [len(flag) - keep], (s, removed, len(flag) - keep)
        # inflow: a layer of new particles just inside the left active face
        k = 100
        xin = np.zeros((3, k))
        xin[0] = g + rng.random(k) * 0.4
        xin[1] = rng.random(k) * n[1]
        xin[2] = rng.random(k) * n[2]
        new_ids = np.arange(next_id, next_id + k, dtype=np.uint64)
        next_id += k
        assert run.inject(0, xin, np.zeros((3, k)), ids=new_ids) == B.PL_OK
        ox = np.concatenate([np.stack(cols[:3])[:, :keep], xin], axis=1)
        oids = np.concatenate([cols[3][:keep], new_ids])
    assert run.sync() == B.PL_OK
    gx, gu, gid, _ = run.state(0)
    assert np.array_equal(gid, oids)
    assert np.abs(gx - ox).max() <= 1e-11
    assert run.items[0].p.n == len(oids)
    # capacity is enforced
    big = np.zeros((3, 2 * npart))
    assert B.pl_part_inject(run.ctx, run.items[0], big.shape[1], [0, 0, 0], [0, 0, 0], cap=2 * npart,
                            check=False) == B.PL_EINVAL
    run.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_boundary_edge_cases(mods, prec):
    """No open dimension: nothing removed, every array untouched.  Every
    particle inside the ghost layers of an open dimension: all removed, and the
    emptied item sorts and steps.  An empty item: nothing removed."""
    oracle, driver, inputs, B = mods
    n = 16
    p = B.PL_F64 if prec == "f64" else B.PL_F32_OFFSET
    say(f"[lp] boundary edge cases {prec}")
    rng = np.random.default_rng(77)
    # nothing open
    wl = inputs.turbulent_box(n=n, npart=777, steps=1)
    run = driver.Run(wl, prec=p, algo=B.PL_ALGO_TILED, tile=(4, 4, 4))
    run.sort()
    before = {k: (np.stack(v) if isinstance(v, list) else v).copy() for k, v in run.raw(0).items()}
    assert run.boundary((0, 0, 0), 2) == [0]
    assert run.items[0].p.n == 777
    after = run.raw(0)
    for k, v in before.items():
        assert np.array_equal(v, np.stack(after[k]) if isinstance(after[k], list) else after[k]), k
    run.step(flags=0)
    assert run.sync() == B.PL_OK
    run.close()
    # every particle in the ghost layers of x (x < 2 or x >= n - 2)
    npart = 500
    x = rng.random((3, npart)) * n
    x[0] = np.where(rng.random(npart) < 0.5, rng.random(npart) * 2.0, n - 2.0 + rng.random(npart) * 1.999)
    wl.items[0].particles = inputs.make_particles(x, np.zeros((3, npart)))
    run = driver.Run(wl, prec=p, algo=B.PL_ALGO_TILED, tile=(4, 4, 4))
    run.sort()
    assert run.boundary((1, 0, 0), 2) == [npart]
    assert run.items[0].p.n == 0
    run.sort()
    run.step(flags=0)
    assert run.sync() == B.PL_OK
    run.close()
    # an empty item
    wl.items[0].particles = inputs.make_particles(np.zeros((3, 0)), np.zeros((3, 0)))
    run = driver.Run(wl, prec=p, algo=B.PL_ALGO_TILED, tile=(4, 4, 4))
    run.sort()
    assert run.boundary((1, 1, 1), 2) == [0]
    assert run.items[0].p.n == 0
    run.close()
