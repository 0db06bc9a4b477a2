"""Strength of the oracle's pins: each test plants one plausible mistake in a copy of the
oracle's source (on the CPU), builds it, and runs the pin suite against that copy through
ORACLE_LIB_OVERRIDE; at least one pin must fail.  Marked slow (about a minute in all)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "reann_oracle.c")

# name: (text in the oracle's source, its planted replacement); each text occurs once
MUTATIONS = {
    "multinomial weights dropped": ("q->w[k] = om_fact(l) / (om_fact(lx) * om_fact(ly) * om_fact(lz));",
                                    "q->w[k] = 1.0;"),
    "cutoff not squared": ("    return u * u;\n", "    return u;\n"),
    "radial derivative sign": ("double dR = -2.0 * m->alphas[mm] * x * R;", "double dR = 2.0 * m->alphas[mm] * x * R;"),
    "centre's message instead of the neighbour's": ("double w = c_ext[e * K + mm] * exp(", "double w = c_ext[a * K + mm] * exp("),
    "no ghost message gather": ("            for (int64_t e = 0; e < Dp->n_ext; ++e)\n                memcpy(c[p][t + 1] + e * K,",
                                "            for (int64_t e = 0; e < Dp->n_loc; ++e)\n                memcpy(c[p][t + 1] + e * K,"),
    "no reverse sum of ghost message adjoints": (
        "                for (int64_t e = 0; e < D[p].n_ext; ++e)\n                    for (int k = 0; k < K; ++k) cbglob[",
        "                for (int64_t e = 0; e < D[p].n_loc; ++e)\n                    for (int k = 0; k < K; ++k) cbglob["),
    "hidden-layer bias dropped": ("            double z = bb[o];\n", "            double z = 0.0;\n"),
    "virial sign": ("W[3 * a + b] -= d[a] * g[b];", "W[3 * a + b] += d[a] * g[b];"),
    "density adjoint misses the symmetric term": ("Sbar[k * K + b] += rb * q->w[k] * S[k * K + a];",
                                                  "if (a != b) Sbar[k * K + b] += rb * q->w[k] * S[k * K + a];"),
    "periodic self-images excluded": ("if (e == i) continue;", "if (e == i || D->gid[e] == D->gid[i]) continue;"),
    "radial gradient not projected on d / r": ("A[l] * radial * d[k] / r);", "A[l] * radial * d[k]);"),
    "message adjoint without the cutoff": ("cb += s * A[l] * R * fc;", "cb += s * A[l] * R;"),
    "energy scale missing in the backward": ("                double rho[1024], rhobar[1024], ybar = m->energy_scale;\n"
                                             "                om_features(m, &C.q, S[p][T - 1]",
                                             "                double rho[1024], rhobar[1024], ybar = 1.0;\n"
                                             "                om_features(m, &C.q, S[p][T - 1]"),
    "radial form without the residual update": ("ci[k] += c[p][t][i * K + k];", "ci[k] += 0.0;"),
    "radial adjoint without the residual": ("for (int64_t x = 0; x < n * K; ++x) cbglob[x] += cbnext[x];",
                                            "for (int64_t x = 0; x < n * K; ++x) cbglob[x] += 0.0 * cbnext[x];"),
    "radial features squared": ("{ memcpy(rho, S, sizeof(double) * K); return; }",
                                "{ for (int k = 0; k < K; ++k) rho[k] = S[k] * fabs(S[k]); return; }"),
    "diag features without the multinomial weights": ("if (q->l[k] == l) s += q->w[k] * S[k * K + a] * S[k * K + a];",
                                                      "if (q->l[k] == l) s += S[k * K + a] * S[k * K + a];"),
    "diag adjoint without the factor 2": ("Sbar[k * K + a] = 2.0 * q->w[k] * S[k * K + a]",
                                          "Sbar[k * K + a] = q->w[k] * S[k * K + a]"),
    "halo one cutoff short": ("rc = om_domain_build(&g, species, p, rcut, T * rcut, 1, &D);",
                              "rc = om_domain_build(&g, species, p, rcut, (T - 1) * rcut, 1, &D);"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", list(MUTATIONS))
def test_a_pin_catches_the_planted_mistake(tmp_path, name):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "the planted text must occur exactly once: %r" % old
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC",
                           "-o", str(lib), str(mut), "-lm"])
    env = dict(os.environ, ORACLE_LIB_OVERRIDE=str(lib), OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_radial.py"),
                        os.path.join(ROOT, "tests", "test_oracle_diag.py")], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-600:]
    assert r.returncode == 1, "no pin failed for the planted mistake %r:\n%s" % (name, tail)
