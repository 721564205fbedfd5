"""Do the oracle's pins catch mistakes?  Each case plants one plausible error
in a copy of oracle/oracle.c (on the CPU only), builds the copy with the
oracle's own flags, and runs the pins of test_oracle.py and
test_oracle_force.py against it in a subprocess: at least one pin must fail.
The unmodified source, built and run the same way, must pass them all."""

import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["tests/test_oracle.py", "tests/test_oracle_force.py"]

# (name, text in oracle.c, planted replacement)
MUTATIONS = [
    ("projector-sign", "cplx p = (s == r ? 1.0 : 0.0) - dir * GAM[mu][s][r];",
     "cplx p = (s == r ? 1.0 : 0.0) + dir * GAM[mu][s][r];"),
    ("no-boundary-phase", "if (wrapped) eta = cexp(I * (dir * M_PI * theta[mu]));",
     "if (wrapped) eta = 1.0;"),
    ("backward-phase-not-conjugated", "if (wrapped) eta = cexp(I * (dir * M_PI * theta[mu]));",
     "if (wrapped) eta = cexp(I * (M_PI * theta[mu]));"),
    ("backward-link-without-dagger", "cplx ub = dir > 0 ? u[3 * a + b] : conj(u[3 * b + a]);",
     "cplx ub = dir > 0 ? u[3 * a + b] : u[3 * a + b];"),
    ("transposed-links", "cplx ub = dir > 0 ? u[3 * a + b] : conj(u[3 * b + a]);",
     "cplx ub = dir > 0 ? u[3 * b + a] : conj(u[3 * a + b]);"),
    ("backward-link-from-output-site", "(dir > 0 ? x : y)", "x"),
    ("wrap-to-wrong-site", "if (d[mu] < 0) { d[mu] = g->L[mu] - 1; *wrapped = 1; }",
     "if (d[mu] < 0) { d[mu] = 0; *wrapped = 1; }"),
    ("kappa-dropped", "out[3 * s + a] = kappa * acc[s][a];", "out[3 * s + a] = acc[s][a];"),
    ("gamma1-entry-sign", "const cplx g1[4][4] = {{0, 0, 0, -i},", "const cplx g1[4][4] = {{0, 0, 0, i},"),
    ("twist-sign-in-A-inverse", "spin_lincomb_g5(te, te, Vh, 1.0 / D, -I * mt / D);         /* A^-1 */",
     "spin_lincomb_g5(te, te, Vh, 1.0 / D, I * mt / D);         /* A^-1 */"),
    ("twist-sign-in-A", "spin_lincomb_g5(te, x, Vh, 1.0, I * mt);",
     "spin_lincomb_g5(te, x, Vh, 1.0, -I * mt);"),
    ("cg-beta-inverted", "const double beta = rr_new / rr;", "const double beta = rr / rr_new;"),
    ("force-trace-kept", "f[3 * a + b] += coeff * (A[a][b] - (a == b ? tr / 3.0 : 0.0));",
     "f[3 * a + b] += coeff * A[a][b];"),
    ("force-hermitian-part", "A[a][b] = 0.5 * (M[a][b] - conj(M[b][a]));",
     "A[a][b] = 0.5 * (M[a][b] + conj(M[b][a]));"),
    ("euclidean-gradient-no-dagger", "f[3 * a + b] += coeff * (forward ? conj(W[b][a]) : W[a][b]);",
     "f[3 * a + b] += coeff * W[a][b];"),
    ("force-backward-sign", "sum += forward ? u[3 * a + k] * W[k][b] : -W[a][k] * conj(u[3 * b + k]);",
     "sum += forward ? u[3 * a + k] * W[k][b] : W[a][k] * conj(u[3 * b + k]);"),
]


def build_variant(tmp_path, text):
    src = tmp_path / "oracle_variant.c"
    src.write_text(text)
    so = tmp_path / "liboracle_variant.so"
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", str(so), str(src), "-lm"])
    return so


def run_pins(so):
    env = dict(os.environ, ORACLE_LIB=str(so), OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        *PINS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    return r.returncode, r.stdout + r.stderr


def source():
    with open(oracle._SRC) as fh:
        return fh.read()


def test_unmodified_copy_passes_the_pins(tmp_path):
    rc, out = run_pins(build_variant(tmp_path, source()))
    assert rc == 0, out[-3000:]


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_fails_a_pin(tmp_path, name, old, new):
    text = source()
    assert text.count(old) == 1, f"mutation site of {name} not unique in oracle.c"
    rc, out = run_pins(build_variant(tmp_path, text.replace(old, new)))
    assert rc == 1, out[-3000:]
