"""The closure and march pins can tell a wrong oracle from the right one.

Each case plants one plausible mistake in a copy of the oracle's source
(on the CPU, in a temporary directory), builds it, and runs the pins of
``test_oracle_closures.py`` against that build in a fresh process: at least
one pin must fail.  The mistakes are those an implementation of Sec. 3 of
the paper could make when it turns tallies into the inputs of the HLOSM
solve or marches the LOSM equations:
  - the sign of F = phi/3 - K (Eq. F) at either time level;
  - the weights of the edge-current interpolation (each cell weighted by its
    own width instead of the opposite one's);
  - the W_start / W_done scale of the closures of a partial step (Eq. Hpn);
  - the time level of the closures F^n or of P^n in the march (Eq.
    losm-disc);
  - the sign of J_0 in the left boundary relation, or the faces of P_L and
    P_R swapped (Eq. losm-disc-bc);
  - the initial condition of an implicit update taken from the step being
    swept instead of the previous time layer;
  - the time-layer tallies normalised like track-length ones (an extra
    1/dt, Eqs. phi-mc and ct-mc).
Not GPU.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "hww_oracle.c")
PINS = os.path.join(ROOT, "tests", "test_oracle_closures.py")

MUTATIONS = {
    "F sign, old level": ("F_o[i] = gi.phi[i - 1] / 3.0 - gi.K[i - 1];",
                          "F_o[i] = gi.K[i - 1] - gi.phi[i - 1] / 3.0;"),
    "F sign, new level": ("F_n[i] = gc.phi[i - 1] / 3.0 - gc.K[i - 1];",
                          "F_n[i] = gc.K[i - 1] - gc.phi[i - 1] / 3.0;"),
    "interpolation weights swapped": ("J_o[i] = (dr * gi.J[i - 1] + dl * gi.J[i]) / (dl + dr);",
                                      "J_o[i] = (dl * gi.J[i - 1] + dr * gi.J[i]) / (dl + dr);"),
    "no W_start/W_done scale": ("scale = bank_weight(s, 1) / nval(&done);", "scale = 1.0;"),
    "march: lagged F": ("F + (size_t)(n - 1) * M, F + (size_t)n * M,",
                        "F + (size_t)(n - 1) * M, F + (size_t)(n - 1) * M,"),
    "march: P of the old level": ("P[2 * n], P[2 * n + 1]", "P[2 * n - 2], P[2 * n - 1]"),
    "J_0 boundary sign": ("J_o[0] = -0.5 * phi_o[0] + gi.fP[0];", "J_o[0] = 0.5 * phi_o[0] + gi.fP[0];"),
    "P_L and P_R swapped": ("P[0] = gi.fP[0]; P[1] = gi.fP[1];", "P[0] = gi.fP[1]; P[1] = gi.fP[0];"),
    "implicit IC from the current step": ("ic = &s->prev; cl = &s->cur;", "ic = &s->cur; cl = &s->cur;"),
    "time-layer tally over dt": ("double norm = track ? (N * dxi * s->dt) : (N * dxi);",
                                 "double norm = N * dxi * s->dt;"),
}


@pytest.fixture(scope="module")
def workdir(tmp_path_factory):
    d = tmp_path_factory.mktemp("oracle_mutants")
    shutil.copy(os.path.join(ROOT, "oracle", "hww_oracle.h"), d)
    return d


def _build(workdir, name, text):
    c = os.path.join(workdir, name + ".c")
    so = os.path.join(workdir, name + ".so")
    with open(c, "w") as f:
        f.write(text)
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC", "-shared",
                    "-I", str(workdir), "-o", so, c, "-lm"], check=True)
    return so


def _run_pins(so):
    env = dict(os.environ, HWW_ORACLE_LIB=so)
    return subprocess.run([sys.executable, "-m", "pytest", PINS, "-q", "-p", "no:cacheprovider"],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


def test_unmutated_copy_passes(workdir):
    with open(SRC) as f:
        text = f.read()
    r = _run_pins(_build(workdir, "clean", text))
    assert r.returncode == 0, r.stdout[-3000:]


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_mutation_fails_a_pin(workdir, name):
    before, after = MUTATIONS[name]
    with open(SRC) as f:
        text = f.read()
    assert text.count(before) == 1, f"mutation site of '{name}' not found once in the oracle"
    r = _run_pins(_build(workdir, "m%d" % list(MUTATIONS).index(name), text.replace(before, after)))
    # A failed assertion (exit 1), not an error of collection or of the build.
    assert r.returncode == 1, r.stdout[-3000:]
    assert " failed" in r.stdout.splitlines()[-1], r.stdout[-3000:]
