"""Planted mistakes in the oracle must each fail at least one of its pins.

Each mutant is the oracle's C source with one plausible slip (a dropped
term, a wrong sign, power or coefficient, a broken tie-break or split),
compiled with gcc into a temporary library.  The pin tests of the part it
touches then run against it in a child process, with NBODY_ORACLE_LIB
pointing the oracle there, and must fail on an assertion.  The pins are
thereby shown to depend on the arithmetic they claim to check."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "nbody_oracle.c")

# (name, pin files, exact text, replacement[, anchor]); the text must occur
# once, or, with an anchor, the first occurrence after the anchor is replaced
MUTANTS = [
    ("force: power 2 instead of 3/2", ["tests/test_oracle_force.py"],
     "const double w = 1.0 / (r2 * r); /* (r^2 + eps^2)^(-3/2) */",
     "const double w = 1.0 / (r2 * r2); /* (r^2 + eps^2)^(-3/2) */"),
    ("force: softening dropped", ["tests/test_oracle_force.py"],
     "const double r2 = ((dx * dx + dy * dy) + dz * dz) + eps2;\n            const double r = sqrt(r2);\n"
     "            const double w = 1.0 / (r2 * r); /*",
     "const double r2 = ((dx * dx + dy * dy) + dz * dz);\n            const double r = sqrt(r2);\n"
     "            const double w = 1.0 / (r2 * r); /*"),
    ("force: sign of one component", ["tests/test_oracle_force.py"],
     "            nsum_add(&ax, mw * dx);\n            nsum_add(&ay, mw * dy);\n            nsum_add(&az, mw * dz);\n"
     "            nsum_add(&ph, m[j] / r);",
     "            nsum_add(&ax, mw * dx);\n            nsum_add(&ay, -mw * dy);\n            nsum_add(&az, mw * dz);\n"
     "            nsum_add(&ph, m[j] / r);"),
    ("force: self pair kept", ["tests/test_oracle_force.py"],
     "        for (int64_t j = 0; j < n; ++j) {\n            if (j == i)\n                continue;\n"
     "            const double dx = x[3 * j] - xi;",
     "        for (int64_t j = 0; j < n; ++j) {\n            const double dx = x[3 * j] - xi;"),
    ("potential: sign", ["tests/test_oracle_force.py"],
     "pot[t] = -G * nsum_val(&ph);\n    }\n}\n\n/* ----", "pot[t] = G * nsum_val(&ph);\n    }\n}\n\n/* ----"),
    ("force: G dropped from one component", ["tests/test_oracle_force.py", "tests/test_oracle_leapfrog.py",
                                             "tests/test_oracle_vjp.py"],
     "acc[3 * t + 1] = G * nsum_val(&ay);\n            acc[3 * t + 2] = G * nsum_val(&az);\n        }\n"
     "        if (pot)\n            pot[t] = -G * nsum_val(&ph);\n    }\n}\n",
     "acc[3 * t + 1] = nsum_val(&ay);\n            acc[3 * t + 2] = G * nsum_val(&az);\n        }\n"
     "        if (pot)\n            pot[t] = -G * nsum_val(&ph);\n    }\n}\n"),
    ("energy: potential energy not halved", ["tests/test_oracle_force.py", "tests/test_oracle_leapfrog.py"],
     "nsum_add(&u, 0.5 * m[i] * pot[i]);", "nsum_add(&u, m[i] * pot[i]);"),
    ("leapfrog: full kicks", ["tests/test_oracle_leapfrog.py"],
     "    const double h = 0.5 * dt;\n    oracle_accel(n, x, m, G, eps, n, NULL, acc, pot);",
     "    const double h = dt;\n    oracle_accel(n, x, m, G, eps, n, NULL, acc, pot);"),
    ("ORB: axis ties to the higher axis", ["tests/test_oracle_orb.py"],
     "    if (ext[1] > ext[axis])\n        axis = 1;", "    if (ext[1] >= ext[axis])\n        axis = 1;"),
    ("ORB: left part rounded down", ["tests/test_oracle_orb.py"],
     "    int64_t k = (int64_t)leaf * ((L + 1) / 2);\n    if (k > cnt)\n        k = cnt;\n"
     "    orb_rec(xf, s, k, leaf, tmp);",
     "    int64_t k = (int64_t)leaf * (L / 2);\n    if (k > cnt)\n        k = cnt;\n"
     "    orb_rec(xf, s, k, leaf, tmp);"),
    ("VJP: coefficient of the d d^T term", ["tests/test_oracle_vjp.py"],
     "nsum_add(&gx, w * e0 - 3.0 * u * d0 * de);", "nsum_add(&gx, w * e0 - 2.0 * u * d0 * de);"),
    ("VJP: sign of the mass cotangent", ["tests/test_oracle_vjp.py"],
     "nsum_add(&gm, -w * da);", "nsum_add(&gm, w * da);"),
    ("VJP: sign of the potential's mass term", ["tests/test_oracle_vjp.py"],
     "nsum_add(&gm, -phibar[j] / r);", "nsum_add(&gm, phibar[j] / r);"),
    ("tree: opening test twice as loose", ["tests/test_oracle_tree.py"],
     "return t->diag2[c] < t->theta2 * D2;", "return t->diag2[c] < 2.0 * t->theta2 * D2;"),
    ("pseudo-particles: quadrupole weight", ["tests/test_oracle_pseudo.py"],
     "t = t + 5.0 / PSEUDO_K * ((3.0 * cj * cj - r2) / (2.0 * a * a));",
     "t = t + 4.0 / PSEUDO_K * ((3.0 * cj * cj - r2) / (2.0 * a * a));"),
    ("quadrupole cells: force coefficient", ["tests/test_oracle_quad.py"],
     "nsum_add(ak, -2.5 * dqd * dv[k] / s7);", "nsum_add(ak, -2.0 * dqd * dv[k] / s7);"),
    ("local expansion: quadrupole part of P0", ["tests/test_oracle_local.py"],
     "nsum_add(&L[0], M * s1 + 0.5 * rqr * s5);", "nsum_add(&L[0], M * s1 + 0.4 * rqr * s5);"),
    ("fixed point: full kicks", ["tests/test_oracle_janus.py"],
     "const double kick_scale = 0.5 * dt * G * ldexp(1.0, sv);",
     "const double kick_scale = dt * G * ldexp(1.0, sv);"),
    ("fixed point: half drifts", ["tests/test_oracle_janus.py"],
     "const double drift_scale = dt * ldexp(1.0, sx - sv);",
     "const double drift_scale = dt * ldexp(1.0, sx - sv - 1);"),
    ("ORB: keys without the index tie-break", ["tests/test_oracle_orb.py"],
     "(uint32_t)s[p];", "(uint32_t)0;"),
    ("local expansion: group size left out of its test", ["tests/test_oracle_local.py"],
     "if (t->diag2[c] + t->diag2[g] < t->theta2 * dz2) {", "if (t->diag2[c] < t->theta2 * dz2) {"),
    ("trajectory gradient: drift adjoint with h", ["tests/test_oracle_vjp.py"],
     "            gv[k] += dt * gx[k];", "            gv[k] += h * gx[k];", "double oracle_traj_grad("),
    ("trajectory cotangents: drift adjoint with h", ["tests/test_oracle_vjp.py"],
     "            gv[k] += dt * gx[k];", "            gv[k] += h * gx[k];", "int oracle_traj_grad_cot("),
    ("trajectory cotangents: VJP at x_0 dropped", ["tests/test_oracle_vjp.py"],
     "    oracle_vjp(n, xs, m, G, eps, carry, NULL, tx, tm);\n    for (size_t k = 0; k < n3; ++k)\n"
     "        gx[k] += tx[k];",
     "    oracle_vjp(n, xs, m, G, eps, carry, NULL, tx, tm);\n    for (size_t k = 0; k < n3; ++k)\n"
     "        gx[k] += 0.0 * tx[k];", "int oracle_traj_grad_cot("),
    ("trajectory cotangents: potential's mass term dropped", ["tests/test_oracle_vjp.py"],
     "            gm[k] += tm[k];\n    }\n    double *carry = a;",
     "            gm[k] += 0.0 * tm[k];\n    }\n    double *carry = a;"),
    ("FMM: L2L drops the T term of the gradient", ["tests/test_oracle_fmm.py"],
     "out[1 + k] = c[1 + k] + kd[k] + 0.5 * tdd[k];", "out[1 + k] = c[1 + k] + kd[k];"),
    ("FMM: acceptance test without the target's size", ["tests/test_oracle_fmm.py"],
     "return d->diag2[a] + d->diag2[b] < f->theta2 * dist2;", "return d->diag2[b] < f->theta2 * dist2;"),
    ("FMM: parent expansion not passed down", ["tests/test_oracle_fmm.py"],
     "tot[20 * c + k] = nsum_val(&own[20 * c + k]) + sh[k];", "tot[20 * c + k] = nsum_val(&own[20 * c + k]);"),
    ("FMM: M2P cells left out of the force", ["tests/test_oracle_fmm.py"],
     "                quad_cell_add(xi, yi, zi, d.com + 3 * b, d.mass[b], Q + 6 * b, eps2, &ax, &ay, &az, &ph);",
     "                (void)b;"),
    ("FMM: M2P offered to inner targets", ["tests/test_oracle_fmm.py"],
     "if (al < 0 && tree_accept(&f->tc, b, a)) {", "if (tree_accept(&f->tc, b, a)) {"),
    ("FMM: self pair kept in P2P", ["tests/test_oracle_fmm.py"],
     "                    if (j == i)\n                        continue;\n                    const double dx = x[3 * j] - xi;\n"
     "                    const double dy = x[3 * j + 1] - yi;\n                    const double dzz",
     "                    const double dx = x[3 * j] - xi;\n"
     "                    const double dy = x[3 * j + 1] - yi;\n                    const double dzz"),
]


@pytest.mark.parametrize("spec", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(tmp_path, spec):
    name, pins, old, new = spec[:4]
    src = open(SRC).read()
    if len(spec) > 4:
        assert src.count(spec[4]) == 1, f"the anchor of mutant '{name}' must occur once in the oracle"
        at = src.index(old, src.index(spec[4]))
        changed = src[:at] + new + src[at + len(old):]
    else:
        assert src.count(old) == 1, f"the text of mutant '{name}' must occur once in the oracle"
        changed = src.replace(old, new)
    mutant = tmp_path / "mutant.c"
    mutant.write_text(changed)
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    "-o", str(lib), str(mutant), "-lm"], check=True, capture_output=True)
    env = dict(os.environ, NBODY_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        *pins], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    # exit status 1: tests ran and one failed (not a crash or a collection error)
    assert r.returncode == 1 and " failed" in r.stdout, \
        f"mutant '{name}' was not caught by {pins} (exit {r.returncode}):\n{r.stdout[-3000:]}"
