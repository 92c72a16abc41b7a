"""The oracle's pins catch the mistakes they are meant to catch.

Each case plants one plausible mistake in a copy of oracle/orc.c, builds it
with the oracle's own flags into a temporary directory, and runs the pins
aimed at that part of the update against it in a child process (ORC_LIB
points the oracle's loader at the copy).  The pins must fail on every
mutant and pass on an unmodified copy built the same way:

* dust: the density channel or the force channel weighted by the charge q
  instead of the mass m (pinned by the dust deposit with q != m, P6, P7, P9);
* charged particles: the force channel weighted by q instead of m, or with a
  factor 2 in its time step (pinned by the Boris identity
  F_p = q w (E_p + vbar x B_p));
* the deposit taken at the old position x^n instead of x^{n+1}, or the
  current from the momentum u instead of the velocity v = u / gamma (pinned by
  the single-particle deposit at the closed-form new position, P4, P8);
* the spectral update (Sec. 2): chi scaled by den instead of den^2, the
  laboratory instead of the proper time step, |B| instead of |B|^2 in the
  magnetic energy density (pinned by the characteristics, number
  conservation, cooling cutoff and proper-time pins);
* the compaction and boundary flags (Sec. 3.2): fillers taken from the end of
  the array backwards instead of in index order, the upper open face one cell late
  (pinned by the holes-and-fillers properties, the flags and the exact
  outflow count).

Nothing here touches the GPU or the HIP library.
"""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "orc.c")

FORCE = "mp[4 + d] = sp->m * wp * (un[d] - uo[d]) / dt;"

# name -> (list of (old text, new text, which occurrence), pins selected by -k)
MUTANTS = {
    "dust_density_from_q": ([("mp[0] = sp->m * wp;", "mp[0] = sp->q * wp;", 0)], "dust_deposit"),
    "dust_force_from_q": ([(FORCE, FORCE.replace("sp->m", "sp->q"), 1)], "dust_deposit"),
    "charged_force_from_q": ([(FORCE, FORCE.replace("sp->m", "sp->q"), 0)], "boris_identity"),
    "charged_force_half": ([(FORCE, FORCE.replace("/ dt;", "/ (2.0 * dt);"), 0)], "boris_identity"),
    "current_from_u": ([("mp[1 + d] = sp->q * wp * v[d];", "mp[1 + d] = sp->q * wp * un[d];", 0)],
                       "time_level"),
    # keep each particle's wrapped old position next to its deposit amounts
    # and deposit there
    "deposit_at_old_position": ([
        ("sizeof(double) * (size_t)(np > 0 ? np : 1) * 8", "sizeof(double) * (size_t)(np > 0 ? np : 1) * 16", 0),
        ("double *mp = mu + 8 * p;", "double *mp = mu + 16 * p;", 0),
        ("for (int k = 0; k < 8; ++k) mp[k] = 0.0;",
         "for (int k = 0; k < 8; ++k) mp[k] = 0.0;\n        for (int d = 0; d < 3; ++d) mp[8 + d] = xp[d];", 0),
        ("double xp[3] = {x[0][p], x[1][p], b->ndim == 3 ? x[2][p] : 0.0};",
         "double xp[3] = {mu[16 * p + 8], mu[16 * p + 9], mu[16 * p + 10]};", 0),
        ("const double *mp = mu + 8 * p;", "const double *mp = mu + 16 * p;", 0),
    ], "time_level"),
    # spectral update (Sec. 2, Eqs. 2-6)
    "spectra_chi_den_unsquared": ([("chi[p * nb + i] * den * den / E;", "chi[p * nb + i] * den / E;", 0)],
                                  "spectra_"),
    "spectra_lab_time": ([("double dtau = dt / gamma_g;", "double dtau = dt;", 0)], "spectra_"),
    "spectra_b_not_squared": ([("par->ub * dot(Bp, Bp)", "par->ub * sqrt(dot(Bp, Bp))", 0)], "spectra_"),
    # holes-and-fillers compaction (Sec. 3.2)
    "compact_fillers_reversed": ([("for (long p = keep; p < np; ++p)", "for (long p = np - 1; p >= keep; --p)", 0)],
                                 "compaction"),
    "outside_upper_face": ([("cell >= (double)(b->n[d] - ghost)", "cell > (double)(b->n[d] - ghost)", 0)],
                           "outside_flags or outflow"),
}

SELECT_ALL = " or ".join(sorted({sel for _, sel in MUTANTS.values()}))


def _replace_nth(text, old, new, nth):
    at = -1
    for _ in range(nth + 1):
        at = text.find(old, at + 1)
        assert at >= 0, f"mutation site not found: {old!r} (occurrence {nth})"
    return text[:at] + new + text[at + len(old):]


def _build(tmp, name, text):
    src = os.path.join(tmp, f"{name}.c")
    so = os.path.join(tmp, f"lib{name}.so")
    with open(src, "w") as f:
        f.write(text)
    shutil.copy(os.path.join(ROOT, "oracle", "orc.h"), tmp)
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                    "-o", so, src, "-lm"], check=True)
    return so


def _pins(so, select):
    env = dict(os.environ, ORC_LIB=so, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_spectra_boundary.py"), "-k", select],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    return r.returncode, r.stdout[-2000:]


@pytest.fixture(scope="module")
def source():
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    with open(SRC) as f:
        return f.read()


def test_unmodified_copy_passes(source, tmp_path):
    rc, out = _pins(_build(str(tmp_path), "orc_copy", source), SELECT_ALL)
    assert rc == 0, out


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_fails_a_pin(source, tmp_path, name):
    edits, select = MUTANTS[name]
    text = source
    for old, new, nth in edits:
        text = _replace_nth(text, old, new, nth)
    assert text != source
    rc, out = _pins(_build(str(tmp_path), name, text), select)
    assert rc == 1, f"{name}: the pins selected by {select!r} did not fail (rc {rc})\n{out}"
