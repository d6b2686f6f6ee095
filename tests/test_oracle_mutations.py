"""The oracle's pins must catch plausible mistakes: each mutant below is a copy of the oracle
with one planted error (compiled on the CPU into a temporary directory), and the pin suite
must fail on every one of them."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lbm_oracle.c")

MUTANTS = {
    "drop_K_in_a3": ("cs2 * (K[a][b] * s[g] + K[b][g] * s[a] + K[g][a] * s[b])",
                     "cs2 * (K[a][b] * s[g] + K[b][g] * s[a])"),
    "h3_sign": ("- L->cs2 * (L->c[i][a] * dbg", "+ L->cs2 * (L->c[i][a] * dbg"),
    "third_order_factor": ("t3 / (6.0 * cs2 * cs2 * cs2)", "t3 / (2.0 * cs2 * cs2 * cs2)"),
    "second_order_factor": ("t2 / (2.0 * cs2 * cs2)", "t2 / (cs2 * cs2)"),
    "stream_backwards": ("int64_t xd = wrap(x + L.c[i][0], nx);", "int64_t xd = wrap(x - L.c[i][0], nx);"),
    "relax_by_tau": ("(feq[i] - fi) / tau", "(feq[i] - fi) * tau"),
    "K_sign": ("K[a][b] = Ainv[a * d + b] - ((a == b) ? 1.0 : 0.0);",
               "K[a][b] = ((a == b) ? 1.0 : 0.0) - Ainv[a * d + b];"),
    "K_transposed_index": ("Ainv[a * d + b] - ((a == b)", "Ainv[a * d + a] - ((a == b)"),
    "theta_without_cs2": ("Ainv[k] = T[k] / cs2;", "Ainv[k] = T[k];"),
    "d3q19_weights": ("(n2 == 1) ? 1.0 / 18.0 : 1.0 / 36.0", "(n2 == 1) ? 1.0 / 12.0 : 1.0 / 48.0"),
    "atilde_sqrt_always": ("double scale = pow(det, 1.0 / d);", "double scale = sqrt(det);"),
    "y_index_swap": ("int64_t yd = wrap(y + L.c[i][1], ny);", "int64_t yd = wrap(y + L.c[i][2], ny);"),
    "bounce_back_same_direction": ("nxt[opp[i] * N + n] = post;", "nxt[i * N + n] = post;"),
    "force_half_missing_in_readout": ("(j[a] + (force ? 0.5 * force[a] : 0.0)) / r", "(j[a] + (force ? force[a] : 0.0)) / r"),
    "force_not_divided_by_rho": ("sf[a] = s[a] + F[a] / rho;", "sf[a] = s[a] + F[a];"),
    "gray_same_direction": ("post = (1.0 - m) * post + m * cur[opp[i] * N + n];",
                            "post = (1.0 - m) * post + m * cur[i * N + n];"),
    "kinetic_energy_factor": ("total += 0.5 * e / r;", "total += e / r;"),
}


@pytest.mark.slow
@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_pins_catch_mutant(mutant):
    old, new = MUTANTS[mutant]
    src = open(SRC).read()
    assert src.count(old) == 1, mutant
    with tempfile.TemporaryDirectory() as tmp:
        c = os.path.join(tmp, "m.c")
        so = os.path.join(tmp, "m.so")
        with open(c, "w") as fh:
            fh.write(src.replace(old, new))
        subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC", c, "-o", so,
                        "-lm"], check=True)
        env = dict(os.environ, LBM_ORACLE_LIB=so, OMP_NUM_THREADS="2")
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                            os.path.join(ROOT, "tests", "test_oracle_walls_force.py"),
                            os.path.join(ROOT, "tests", "test_oracle_gray.py"),
                            os.path.join(ROOT, "tests", "test_oracle_bruteforce.py")], cwd=ROOT, env=env,
                           capture_output=True, text=True, timeout=600)
        assert r.returncode != 0, f"mutant {mutant} survived the pins:\n{r.stdout[-2000:]}"


# mutants of the periodic update, forced or not, that the brute-force transcription alone must
# catch (tensor forms, walls, gray cells and objectives lie outside what it transcribes)
BRUTE_FORCE_SCOPE = ["K_sign", "K_transposed_index", "d3q19_weights", "drop_K_in_a3", "force_half_missing_in_readout",
                     "force_not_divided_by_rho", "h3_sign", "relax_by_tau", "second_order_factor", "stream_backwards",
                     "third_order_factor", "y_index_swap"]


@pytest.mark.slow
@pytest.mark.parametrize("mutant", BRUTE_FORCE_SCOPE)
def test_bruteforce_transcription_alone_catches_mutant(mutant):
    old, new = MUTANTS[mutant]
    src = open(SRC).read()
    with tempfile.TemporaryDirectory() as tmp:
        c = os.path.join(tmp, "m.c")
        so = os.path.join(tmp, "m.so")
        with open(c, "w") as fh:
            fh.write(src.replace(old, new))
        subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC", c, "-o", so,
                        "-lm"], check=True)
        env = dict(os.environ, LBM_ORACLE_LIB=so, OMP_NUM_THREADS="2")
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            os.path.join(ROOT, "tests", "test_oracle_bruteforce.py")], cwd=ROOT, env=env,
                           capture_output=True, text=True, timeout=600)
        assert r.returncode != 0, f"mutant {mutant} survived the brute-force transcription:\n{r.stdout[-2000:]}"
