"""Pins of the oracle's Lagrangian spectral update (Sec. 2, Eqs. cr_N to
cr_chi with the losses of Eq. rad_losses) and of its open-boundary deletion
and holes-and-fillers compaction (Sec. 3.2), against facts fixed outside it:
independent ODE solves of the characteristic equations, the paper's printed
initial spectrum (Sec. 4.2), conservation of particle number in energy space,
invariance of a power law's index under adiabatic change, the cooling cutoff,
composition of steps, and for the compaction the properties that fix its
result uniquely, plus the exact outflow count of a uniform flow.
"""

import math

import numpy as np
import pytest
from scipy import integrate

from paper_2602_23434_amd import inputs


# ---------------------------------------------------------------- spectra

def _uniform_box(n, B=(0.0, 0.0, 0.0), vg=(0.0, 0.0, 0.0), divu=0.0):
    f = inputs.uniform_fields(n, B=B, vg=vg)
    nx, ny, nz = n
    return {"B": f["B"], "vg": f["vg"]}, np.full((nz, ny, nx), float(divu))


def _ode(a, b, eps0, tau):
    """eps and chi / chi0 after proper time tau from the characteristic
    equations of Eq. cr_chi: d eps/d tau = -a eps - b eps^2 and
    d ln chi / d tau = -d(d eps/d tau)/d eps = a + 2 b eps."""
    sol = integrate.solve_ivp(lambda t, y: [-a * y[0] - b * y[0] ** 2, a + 2 * b * y[0]], (0.0, tau),
                              [eps0, 0.0], method="DOP853", rtol=1e-13, atol=1e-15 * eps0)
    return sol.y[0, -1], math.exp(sol.y[1, -1])


@pytest.mark.parametrize("divu,b", [(0.9, 1e-4), (-0.6, 1e-4), (0.0, 1e-3), (1.5, 0.0), (-1.2, 0.0),
                                    (3e-9, 2e-4)])
def test_spectra_characteristics_against_ode(orc, divu, b):
    """Each spectral point follows d eps/d tau = -(div u/3) eps - c_r eps^2
    and chi its Jacobian, to the accuracy of an independent ODE solve."""
    dt = 0.3
    eps0 = np.array([1e2, 7e2, 3e3, 1e4])
    n = (4, 4, 4)
    flds, dv = _uniform_box(n, divu=divu)
    eng = eps0.reshape(1, -1).copy()
    chi = np.full_like(eng, 2.5)
    orc.spectra_step(3, n, 2, np.array([[2.5], [2.5], [2.5]]), flds, dv, eng, chi, dt, cr=1.0, u_rad=b, ub=0.0)
    for i, e0 in enumerate(eps0):
        e_ref, g_ref = _ode(divu / 3.0, b, e0, dt)
        assert abs(eng[0, i] - e_ref) <= 1e-10 * e_ref, (i, eng[0, i], e_ref)
        assert abs(chi[0, i] - 2.5 * g_ref) <= 1e-10 * 2.5 * g_ref, (i, chi[0, i], 2.5 * g_ref)


def test_spectra_number_conserved_along_characteristics(orc):
    """chi d eps is carried unchanged: chi1 * d eps1/d eps0 = chi0, with the
    derivative of the energy map taken by central differences of the oracle
    itself (independent of its chi formula)."""
    n = (4, 4, 4)
    flds, dv = _uniform_box(n, divu=0.45)
    x = np.array([[1.5], [1.5], [1.5]])
    for e0 in (1e2, 2e3, 1e4):
        h = 1e-5 * e0
        eng = np.array([[e0 - h, e0, e0 + h]])
        chi = np.ones_like(eng)
        orc.spectra_step(3, n, 2, x, flds, dv, eng, chi, 0.7, cr=1.0, u_rad=3e-4, ub=0.0)
        jac = (eng[0, 2] - eng[0, 0]) / (2 * h)
        assert abs(chi[0, 1] * jac - 1.0) < 1e-8, (e0, chi[0, 1] * jac)


def test_paper_initial_spectrum():
    """Sec. 4.2's initial spectrum: 128 points from 1e2 to 1e4, index 9, the
    power law integrating to N_0 = 1e-6 over [eps_min, eps_max]."""
    eng, chi = inputs.powerlaw_spectrum()
    assert eng.shape == (128,) and eng[0] == pytest.approx(1e2, rel=1e-15) and eng[-1] == pytest.approx(1e4, rel=1e-15)
    assert np.allclose(np.diff(np.log(eng)), math.log(100.0) / 127, rtol=1e-12)
    slope = np.polyfit(np.log(eng), np.log(chi), 1)[0]
    assert abs(slope + 9.0) < 1e-10
    k = chi[0] * eng[0] ** 9
    total, _ = integrate.quad(lambda e: k * e ** -9.0, 1e2, 1e4, epsrel=1e-13, points=[2e2, 5e2, 1e3])
    assert abs(total - 1e-6) < 1e-12 * 1e-6 * 1e6


def test_spectra_adiabatic_keeps_power_law_and_number(orc):
    """Pure adiabatic change (no losses): a power law keeps its index, and
    the trapezoid number sum_i (chi_i + chi_i+1)/2 (eps_i+1 - eps_i) is
    unchanged (the energy map is a uniform scaling)."""
    eng0, chi0 = inputs.powerlaw_spectrum()
    n = (4, 4, 4)
    for divu in (0.8, -0.5):
        flds, dv = _uniform_box(n, divu=divu)
        eng = eng0.reshape(1, -1).copy()
        chi = chi0.reshape(1, -1).copy()
        orc.spectra_step(3, n, 2, np.array([[0.5], [3.5], [2.0]]), flds, dv, eng, chi, 0.4, cr=1.0, u_rad=0.0,
                         ub=0.0)
        slope = np.polyfit(np.log(eng[0]), np.log(chi[0]), 1)[0]
        assert abs(slope + 9.0) < 1e-9
        trap = lambda e, c: float(np.sum(0.5 * (c[1:] + c[:-1]) * np.diff(e)))
        assert abs(trap(eng[0], chi[0]) - trap(eng0, chi0)) <= 1e-12 * trap(eng0, chi0)
        # compression (div u < 0) heats, expansion cools
        assert (eng[0] > eng0).all() if divu < 0 else (eng[0] < eng0).all()


def test_spectra_cooling_cutoff(orc):
    """Radiative losses alone: eps(tau) = eps0 / (1 + c_r eps0 tau), so no
    energy exceeds 1 / (c_r tau) and the highest energies pile up below it."""
    n = (4, 4, 4)
    flds, dv = _uniform_box(n, divu=0.0)
    b, dt = 2e-4, 0.5
    eng = np.array([[1e2, 1e4, 1e8, 1e14]])
    chi = np.ones_like(eng)
    orc.spectra_step(3, n, 2, np.array([[2.0], [2.0], [2.0]]), flds, dv, eng, chi, dt, cr=1.0, u_rad=b, ub=0.0)
    cut = 1.0 / (b * dt)
    assert (eng[0] < cut).all()
    assert abs(eng[0, -1] - cut) < 1e-9 * cut
    assert abs(eng[0, 0] - 1e2 / (1 + b * 1e2 * dt)) < 1e-12 * 1e2


def test_spectra_steps_compose(orc):
    """With the fluid frozen, two steps of dt/2 equal one step of dt."""
    n = (4, 4, 4)
    flds, dv = _uniform_box(n, divu=-0.7)
    eng0, chi0 = inputs.powerlaw_spectrum(nb=16)
    x = np.array([[2.5], [1.5], [0.5]])
    one_e, one_c = eng0.reshape(1, -1).copy(), chi0.reshape(1, -1).copy()
    orc.spectra_step(3, n, 2, x, flds, dv, one_e, one_c, 0.6, cr=1.0, u_rad=5e-4, ub=0.0)
    two_e, two_c = eng0.reshape(1, -1).copy(), chi0.reshape(1, -1).copy()
    for _ in range(2):
        orc.spectra_step(3, n, 2, x, flds, dv, two_e, two_c, 0.3, cr=1.0, u_rad=5e-4, ub=0.0)
    assert np.allclose(one_e, two_e, rtol=1e-13, atol=0)
    assert np.allclose(one_c, two_c, rtol=1e-12, atol=0)


def test_spectra_proper_time(orc):
    """d tau = dt / gamma_g: in a uniform flow of speed 0.6 c (gamma_g = 1.25)
    a pure adiabatic step scales energies by exp(-(div u/3) dt / 1.25)."""
    n = (4, 4, 4)
    flds, dv = _uniform_box(n, vg=(0.36, 0.0, 0.48), divu=0.9)
    eng = np.array([[1e3]])
    chi = np.ones_like(eng)
    orc.spectra_step(3, n, 2, np.array([[2.5], [2.5], [2.5]]), flds, dv, eng, chi, 0.5, cr=1.0, u_rad=0.0, ub=0.0)
    assert abs(eng[0, 0] - 1e3 * math.exp(-0.3 * 0.5 / 1.25)) < 1e-12 * 1e3


def test_spectra_samples_fields_at_the_particle(orc):
    """The adiabatic rate comes from div u at the particle and the loss rate
    from |B|^2 there: a linear div u field (reproduced exactly by TSC away
    from the seam) and a uniform B of |B|^2 = 4 with U_B = |B|^2 / 2 give, per
    particle, the ODE solution with a = div u(x)/3 and
    b = cr (2 + u_rad)."""
    n = (16, 16, 16)
    nx, ny, nz = n
    xs = np.arange(nx) + 0.5
    dv = np.broadcast_to(0.05 * (xs - 8.0), (nz, ny, nx)).copy()
    f = inputs.uniform_fields(n, B=(0.0, 2.0, 0.0))
    flds = {"B": f["B"], "vg": f["vg"]}
    x = np.array([[3.2, 7.9, 12.4], [5.0, 9.0, 2.0], [8.0, 1.5, 14.0]])
    eng = np.full((3, 2), 1.0) * np.array([3e2, 5e3])
    chi = np.ones_like(eng)
    cr, u_rad, dt = 1e-4, 0.5, 0.8
    orc.spectra_step(3, n, 2, x, flds, dv, eng, chi, dt, cr=cr, u_rad=u_rad, ub=0.5)
    for p in range(3):
        a = 0.05 * (x[0, p] - 8.0) / 3.0
        for i, e0 in enumerate((3e2, 5e3)):
            e_ref, g_ref = _ode(a, cr * (2.0 + u_rad), e0, dt)
            assert abs(eng[p, i] - e_ref) <= 1e-10 * e_ref
            assert abs(chi[p, i] - g_ref) <= 1e-10 * g_ref


# ---------------------------------------------------------------- open boundaries

def test_outside_flags(orc):
    """Active cells [g, n - g) in open dimensions only; positions in cell
    units, a cell is half-open."""
    n = (16, 8, 4)
    g = 2
    x = np.array([[1.999, 2.0, 13.999, 14.0, 0.5, 15.5, 8.0, 8.0],
                  [4.0, 4.0, 4.0, 4.0, 4.0, 4.0, 0.5, 7.9],
                  [1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0]])
    got = orc.outside(3, n, (1, 0, 0), g, x)
    assert got.tolist() == [1, 0, 0, 1, 1, 1, 0, 0]
    got = orc.outside(3, n, (1, 1, 0), g, x)
    assert got.tolist() == [1, 0, 0, 1, 1, 1, 1, 1]
    got = orc.outside(3, n, (0, 0, 0), g, x)
    assert not got.any()


def _check_compaction(flag, ids_before, ids_after, keep, payload_before, payload_after):
    n = len(flag)
    survivors = np.nonzero(flag == 0)[0]
    assert keep == len(survivors)
    got = ids_after[:keep]
    # every survivor exactly once, nothing deleted survives
    assert np.array_equal(np.sort(got), np.sort(ids_before[survivors]))
    # survivors already in the kept prefix do not move
    stay = np.nonzero(flag[:keep] == 0)[0]
    assert np.array_equal(got[stay], ids_before[stay])
    # the holes of the prefix, in increasing order, receive the fillers of the
    # tail in increasing order
    holes = np.nonzero(flag[:keep] != 0)[0]
    fillers = keep + np.nonzero(flag[keep:] == 0)[0]
    assert len(holes) == len(fillers)
    assert np.array_equal(got[holes], ids_before[fillers])
    # every array moved with its particle
    order = np.argsort(ids_before)
    src = order[np.searchsorted(ids_before[order], got)]
    for pb, pa in zip(payload_before, payload_after):
        assert np.array_equal(pa[:keep], pb[src])


@pytest.mark.parametrize("case", ["random", "none", "all", "tail", "head", "one", "empty", "single"])
def test_compaction_holes_and_fillers(orc, case):
    rng = np.random.default_rng(77)
    n = {"empty": 0, "single": 1}.get(case, 1000)
    flag = {"random": (rng.random(n) < 0.3), "none": np.zeros(n, bool), "all": np.ones(n, bool),
            "tail": np.arange(n) >= n - 123, "head": np.arange(n) < 77, "one": np.arange(n) == 500,
            "empty": np.zeros(0, bool), "single": np.ones(1, bool)}[case].astype(np.uint8)
    ids = np.arange(n, dtype=np.uint64) * 7 + 3
    x = rng.random(n)
    cells = rng.integers(0, 1 << 30, n).astype(np.uint32)
    vec = rng.random((n, 3)).astype(np.float32)
    before = [ids.copy(), x.copy(), cells.copy(), vec.copy()]
    keep, holes, fills = orc.compact(flag, [ids, x, cells, vec])
    _check_compaction(flag, before[0], ids, keep, before[1:], [x, cells, vec])
    assert (holes < keep).all() and (fills >= keep).all()
    assert len(holes) == int(flag[:keep].sum())


def test_outflow_of_a_uniform_flow(orc):
    """Tracers in the uniform flow v = 0.3 (cells per unit time along x) of a
    box open in x (two ghost cells each side): after k steps of the tracer
    scheme plus deletion, the survivors are exactly the particles whose
    straight path x0 + k dt v is still inside the active cells."""
    n = (32, 8, 8)
    g = 2
    rng = np.random.default_rng(5)
    npart = 4000
    x = np.zeros((3, npart))
    x[0] = g + rng.random(npart) * (n[0] - 2 * g)
    x[1] = rng.random(npart) * n[1]
    x[2] = rng.random(npart) * n[2]
    u = np.zeros((3, npart))
    ids = np.arange(npart, dtype=np.uint64)
    x0 = x[0].copy()
    f = inputs.uniform_fields(n, vg=(0.3, 0.0, 0.0))
    dt = 1.0
    alive = npart
    for k in range(1, 41):
        xs = np.ascontiguousarray(x[:, :alive])
        us = np.ascontiguousarray(u[:, :alive])
        orc.step(3, n, 2, (2, 0.0, 1.0, 0.0), xs, us, None, {"vg": f["vg"]}, dt)
        flag = orc.outside(3, n, (1, 0, 0), g, xs)
        cols = [np.ascontiguousarray(xs[d]) for d in range(3)] + [np.ascontiguousarray(ids[:alive])]
        keep, _, _ = orc.compact(flag, cols)
        for d in range(3):
            x[d, :keep] = cols[d][:keep]
        ids[:keep] = cols[3][:keep]
        alive = keep
        # exact crossing criterion, away from round-off at the face
        path = x0 + k * dt * 0.3
        clear = np.abs(path - (n[0] - g)) > 1e-9
        expect = set(np.nonzero((path < n[0] - g) & clear)[0].tolist())
        got = set(ids[:alive].tolist())
        assert expect <= got and len(got - expect) <= int((~clear).sum()), k
    assert 0 < alive < npart
