"""Strength of the oracle's pins: each test builds a copy of the oracle's C
source with one plausible mistake planted (a dropped factor, a wrong sign, a
missing normaliser, a transposed index), loads it in place of the oracle and
expects at least one of the pins written for that function to fail.  The
real oracle passes the same pins (``test_oracle_proposal.py`` and the pins of
``test_oracle_pins.py``).  CPU only: nothing here touches the GPU path.
"""
import os
import subprocess

import pytest

import oracle
import proposal_pins as PP

SRC = os.path.join(os.path.dirname(oracle.__file__), "qrfs_oracle.c")

# (name, exact text in the oracle, replacement, pins expected to catch it)
MUTATIONS = [
    ("table: angle of the mixture without the half",
     "phi[j] = 0.5 * atan2(B[j], A[j]);", "phi[j] = atan2(B[j], A[j]);", PP.TABLE_PINS),
    ("table: per-baseline normaliser Z_b dropped",
     "double pj = exp(o0[j] - mx) / Z;", "double pj = exp(o0[j] - mx) * Lw;", PP.TABLE_PINS),
    ("table: cos 2 theta_b replaced by cos theta_b",
     "A[j] += pj * al * cos(2.0 * bth[b]) / (double)nB;",
     "A[j] += pj * al * cos(bth[b]) / (double)nB;", PP.TABLE_PINS),
    ("table: sin and cos swapped in the mixture",
     "B[j] += pj * al * sin(2.0 * bth[b]) / (double)nB;",
     "B[j] += pj * al * cos(2.0 * bth[b]) / (double)nB;", PP.TABLE_PINS),
    ("table: alpha without the 0.9 bound",
     "double al = 0.9 * tanh(o1[j]);", "double al = tanh(o1[j]);", PP.TABLE_PINS),
    ("table: defensive share on the wrong side",
     "p[j] = (1.0 - beta) * pb[j] + beta / Lw;", "p[j] = beta * pb[j] + (1.0 - beta) / Lw;",
     PP.TABLE_PINS),
    ("table: cdf includes its own cell",
     "cdf[j] = run;\n        run += p[j] * dl;", "run += p[j] * dl;\n        cdf[j] = run;",
     PP.TABLE_PINS),
    ("loss: log Z without the cell width",
     "double logZ = mx + log(se * Lw / G);", "double logZ = mx + log(se);", PP.LOSS_PINS),
    ("loss: grid at cell edges instead of midpoints",
     "mlp_features(lmin + (j + 0.5) * Lw / G, lmin, Lw, cc, x);\n            mlp_row(prm, Hd, x, h1, h2, o);\n            og[j] = o[0];",
     "mlp_features(lmin + j * Lw / G, lmin, Lw, cc, x);\n            mlp_row(prm, Hd, x, h1, h2, o);\n            og[j] = o[0];",
     PP.LOSS_PINS),
    ("loss: angular factor with cos(theta - theta_B)",
     "double C = cos(2.0 * (theta[i] - cc[3]));", "double C = cos(theta[i] - cc[3]);",
     PP.LOSS_PINS),
    ("loss: wrong sign of the normaliser",
     "loss -= wi * (o[0] - logZ + log(1.0 + alpha * C));",
     "loss -= wi * (o[0] + logZ + log(1.0 + alpha * C));", PP.LOSS_PINS),
    ("loss: weights not normalised by the total contribution",
     "double wi = h[i] / Htot;", "double wi = h[i] / (double)m;", PP.LOSS_PINS),
]


@pytest.fixture(scope="module")
def source():
    with open(SRC) as f:
        return f.read()


@pytest.mark.parametrize("name,old,new,pins", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(tmp_path, monkeypatch, source, name, old, new, pins):
    assert source.count(old) == 1, f"mutation site not unique: {old!r}"
    src = tmp_path / "mutant.c"
    src.write_text(source.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O1", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                           "-fvisibility=hidden", "-o", str(lib), str(src), "-lm"])
    monkeypatch.setattr(oracle, "_LIB_PATH", str(lib))
    monkeypatch.setattr(oracle, "_lib", None)
    caught = []
    for pin in pins:
        try:
            pin()
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, f"no pin catches: {name}"


def test_real_oracle_passes_the_same_pins():
    for pin in PP.TABLE_PINS + PP.LOSS_PINS:
        pin()
