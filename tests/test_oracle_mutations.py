"""Planted mistakes in the CPU oracle must each be caught by the pins.

Each case copies oracle/bq_oracle.c to a temporary directory, applies one
plausible mistake (a flipped sign, a dropped term, a wrong index, a missing
adjoint, a dropped leaf, a transposed link, a wrong power of kappa), compiles it
with gcc and runs the pins (tests/test_oracle_pins.py, tests/test_oracle_solver_pins.py)
against that build.  The pins must fail for every mutation.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "bq_oracle.c")

MUTATIONS = {
    "forward projector sign": ("mu, -1.0, coef_fwd(L, i, mu, t_bc, mu_ch), nb[mu][0]",
                               "mu, +1.0, coef_fwd(L, i, mu, t_bc, mu_ch), nb[mu][0]"),
    "backward link not daggered": ("link(U, V, mu, b), 1, mu, +1.0", "link(U, V, mu, b), 0, mu, +1.0"),
    "chemical potential sign": ("return exp(mu_ch) *", "return exp(-mu_ch) *"),
    "time boundary sign dropped": ("return exp(-mu_ch) * (x[3] == 0 ? (double)t_bc : 1.0);",
                                   "return exp(-mu_ch) * 1.0;"),
    "trace subtraction dropped": ("Fh[0] -= tr; Fh[4] -= tr; Fh[8] -= tr;", ""),
    "field strength normalisation": ("conj(Q[b * 3 + a])) / 8.0", "conj(Q[b * 3 + a])) / 4.0"),
    "leaf orientation": ("Fh[a * 3 + b] = -I * (Q", "Fh[a * 3 + b] = I * (Q"),
    "second leaf wrong site": ("m3_dag(link(U, V, mu, xpn_mm), A)", "m3_dag(link(U, V, mu, xpn), A)"),
    "dagger hop coefficient": ("conj(coef_bwd(L, f, mu, t_bc, mu_ch))", "conj(coef_fwd(L, f, mu, t_bc, mu_ch))"),
    "clover adjoint transposed": ("(adj ? conj(A[k * NSC + r])", "(adj ? conj(A[r * NSC + k])"),
    "Schur sign": ("out[i * NSC + k] -= kappa * kappa * a[i * NSC + k]", "out[i * NSC + k] += kappa * kappa * a[i * NSC + k]"),
    "source preparation sign": ("b[i * NSC + k] + kappa * c[i * NSC + k] : 0.0", "b[i * NSC + k] - kappa * c[i * NSC + k] : 0.0"),
    "cg residual update": ("r[k] -= alpha * Ap[k];", "r[k] -= alpha * q[k];"),
    "noise imaginary bit": ("(z >> 62) & 1", "(z >> 61) & 1"),
    "hop accumulates by assignment": ("out[s * 3 + a] += coef * acc;", "out[s * 3 + a] = coef * acc;"),
    "dropped clover leaf": ("m3_mul(P, link(U, V, nu, xmn), P);\n    for (int k = 0; k < 9; k++) Q[k] += P[k];",
                            "m3_mul(P, link(U, V, nu, xmn), P);"),
    "transposed forward link": ("cplx w = W_dag ? conj(W[b * 3 + a]) : W[a * 3 + b];",
                                "cplx w = W_dag ? conj(W[b * 3 + a]) : W[b * 3 + a];"),
    "wrong kappa power in the Schur form": ("out[i * NSC + k] -= kappa * kappa * a[i * NSC + k]",
                                            "out[i * NSC + k] -= kappa * a[i * NSC + k]"),
    "dD/dmu backward sign": ("-coef_bwd(L, i, 3, t_bc, mu_ch), in + b * NSC",
                             "coef_bwd(L, i, 3, t_bc, mu_ch), in + b * NSC"),
    "sigma F plane order": ("Si[(s * 3 + a) * NSC + t * 3 + b] += SIG[mu][nu][s][t] * Fh[a * 3 + b];",
                            "Si[(s * 3 + a) * NSC + t * 3 + b] += SIG[nu][mu][s][t] * Fh[a * 3 + b];"),
}
PIN_FILES = ("test_oracle_pins.py", "test_oracle_solver_pins.py")


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_mutation(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor not found: {old!r}"
    mutated = src.replace(old, new, 1)
    c = tmp_path / "bq_oracle.c"
    c.write_text(mutated)
    lib = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-w", "-o", str(lib), str(c), "-lm"],
                   check=True)
    env = dict(os.environ, BQ_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *[os.path.join(ROOT, "tests", f) for f in PIN_FILES]],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutation '{name}' survived the pins:\n{r.stdout[-2000:]}"
