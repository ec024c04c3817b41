"""Mutation check of the oracle's pins: each case plants one plausible mistake
in a copy of the oracle sources (on the CPU, in a temporary directory), builds
that copy and runs the pin suites against it; at least one pin must fail.

The mistakes are the ones a reader of the algorithms could plausibly make:
a threshold compared against theta instead of theta / 2, strict instead of
inclusive comparisons, an off-by-one count of dumped directions, a residual
that is not downdated, a wrong Philox key for a level's FD reduce, a wrong
level threshold, and in the persistent oracle a wrong shrink threshold index
or a missing power step; in the ATTP oracle a historical filter that
drops the snapshot taken at time t, a wrong or stale threshold, the
residual added to past times, a wrong Philox key and a wrong restore sign;
in the probability amplification the candidate with the largest estimate
kept, the smallest of the power iterations taken, the residual not formed,
and a wrong start-vector counter; in P5 the listing's unscaled site
threshold, a counter not reset after its message, a broadcast at every
message or to all sites but one, a wrong restore sign and a wrong key of a
site's FD reduce; in AeroSketchCOD a wrong reduce index, firing at theta,
dumping by squared values, a strict expiry, a B side not downdated and a wrong
restore sign.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")

# (file, original text, mutated text, pin files expected to catch it)
WINDOW_PINS = ["tests/test_oracle_window_pins.py", "tests/test_oracle_window.py"]
FD_PINS = ["tests/test_oracle_pins.py"]
ATTP_PINS = ["tests/test_oracle_attp.py"]
AMP_PINS = ["tests/test_oracle_amplify.py"]
P5_PINS = ["tests/test_oracle_p5.py"]
COD_PINS = ["tests/test_oracle_cod.py"]
MUTANTS = {
    "pi_threshold_theta": ("window.c", "if (!(s1 >= theta / 2.0)) return 0;",
                           "if (!(s1 >= theta)) return 0;", WINDOW_PINS),
    "pi_threshold_strict": ("window.c", "if (!(s1 >= theta / 2.0)) return 0;",
                            "if (!(s1 > theta / 2.0)) return 0;", WINDOW_PINS),
    "xi_strict": ("window.c", "while (xi < k && est[xi] >= theta) ++xi;",
                  "while (xi < k && est[xi] > theta) ++xi;", WINDOW_PINS),
    "xi_plus_one": ("window.c", "while (xi < k && est[xi] >= theta) ++xi;",
                    "while (xi < k && est[xi] >= theta) ++xi;\n            if (xi > 0 && xi < k) ++xi;",
                    WINDOW_PINS),
    "xi_minus_one": ("window.c", "while (xi < k && est[xi] >= theta) ++xi;",
                     "while (xi < k && est[xi] >= theta) ++xi;\n            if (xi > 1) --xi;", WINDOW_PINS),
    "no_residual_downdate": ("window.c", "C[rr * d + t] -= acc;", "C[rr * d + t] -= 0.0 * acc;",
                             WINDOW_PINS),
    "raw_strict": ("window.c", "if (nrm >= l->theta) {", "if (nrm > l->theta) {", WINDOW_PINS),
    "level_key": ("window.c", "w->stream * 64u + (uint64_t)j + 1u", "w->stream * 64u + (uint64_t)j",
                  WINDOW_PINS),
    "level_theta": ("window.c", "l->theta = ldexp(1.0, j) * eps * (double)N;",
                    "l->theta = ldexp(1.0, j + 1) * eps * (double)N;", WINDOW_PINS),
    "exact_delta_index": ("fd.c", "double delta = (m >= ell) ? sigma[ell - 1] * sigma[ell - 1] : 0.0;",
                          "double delta = (m > ell) ? sigma[ell] * sigma[ell] : 0.0;", FD_PINS),
    "rand_delta_index": ("fd.c", "double delta = (k >= ell) ? fmax(w[ell - 1], 0.0) : 0.0;",
                         "double delta = (k > ell) ? fmax(w[ell], 0.0) : fmax(w[k - 1], 0.0);", FD_PINS),
    "rand_power_step_dropped": ("fd.c", "for (int it = 0; it < q; ++it) {", "for (int it = 1; it < q; ++it) {",
                                FD_PINS),
    "rand_omega_shrink_counter": ("fd.c", "o_omega(seed, stream, b, 0, d, k, Om);",
                                  "o_omega(seed, stream, 0, 0, d, k, Om);", FD_PINS),
    "fill_after_shrink": ("fd.c", "s->r = s->ell - 1;", "s->r = s->ell;", FD_PINS),
    "attp_history_strict": ("attp.c", "if (s->t > t) continue;", "if (s->t >= t) continue;", ATTP_PINS),
    "attp_theta_eps": ("attp.c", "a->theta = (2.0 / ell) * a->fro2;", "a->theta = (1.0 / ell) * a->fro2;",
                       ATTP_PINS),
    "attp_theta_stale": ("attp.c", "a->fro2 += nrm;\n    a->theta = (2.0 / ell) * a->fro2;",
                         "a->theta = (2.0 / ell) * a->fro2;\n    a->fro2 += nrm;", ATTP_PINS),
    "attp_residual_in_history": ("attp.c", "if (t == a->T)", "if (t >= 0)", ATTP_PINS),
    "attp_reduce_key": ("attp.c", "a->stream * 64u + 1u", "a->stream * 64u", ATTP_PINS),
    "attp_restore_sign": ("attp.c", "G[(int64_t)x * d + y] += acc - sub;", "G[(int64_t)x * d + y] += acc + sub;",
                          ATTP_PINS),
    "amp_keeps_largest": ("window.c", "if (besth < 0 || ch < best) {", "if (besth < 0 || ch > best) {", AMP_PINS),
    "amp_min_over_power_iterations": ("window.c", "if (e > ch) ch = e;", "if (g == 0 || e < ch) ch = e;", AMP_PINS),
    "amp_no_residual": ("window.c", "R[rr * d + t] -= cz * Zh[(int64_t)t * k + c];",
                        "R[rr * d + t] -= 0.0 * cz * Zh[(int64_t)t * k + c];", AMP_PINS),
    "amp_power_counter": ("window.c", "0x100000u + 0x10000u * (uint64_t)g", "0x100000u + 0x10000u * (uint64_t)(g + 1)",
                          AMP_PINS),
    "p5_site_threshold_unscaled": ("p5.c", "const double theta = (eps / m) * s->Fhat;",
                                   "const double theta = eps * s->Fhat;", P5_PINS),
    "p5_counter_not_reset": ("p5.c", "p->Fhat += s->F;\n        s->F = 0.0;", "p->Fhat += s->F;", P5_PINS),
    "p5_broadcast_every_message": ("p5.c", "if (p->nmsg >= m) {", "if (p->nmsg >= 1) {", P5_PINS),
    "p5_broadcast_skips_a_site": ("p5.c", "for (int k = 0; k < m; ++k) p->s[k].Fhat = p->Fhat;",
                                  "for (int k = 1; k < m; ++k) p->s[k].Fhat = p->Fhat;", P5_PINS),
    "p5_restore_sign": ("p5.c", "p->B[(int64_t)x * d + y] += acc - sub;", "p->B[(int64_t)x * d + y] += acc + sub;",
                        P5_PINS),
    "p5_site_reduce_key": ("p5.c", "sid * 64u + 1u", "sid * 64u", P5_PINS),
    "cod_reduce_index": ("cod.c", "const double delta = (p >= ell) ? s[ell - 1] : 0.0;\n        memset(A",
                         "const double delta = (p > ell) ? s[ell] : 0.0;\n        memset(A", COD_PINS),
    "cod_fire_at_theta": ("cod.c", "if (s1 >= c->theta / 2.0) {", "if (s1 >= c->theta) {", COD_PINS),
    "cod_dump_squared": ("cod.c", "while (xi < k && sqrt(fmax(eh[xi], 0.0)) >= c->theta) ++xi;",
                         "while (xi < k && fmax(eh[xi], 0.0) >= c->theta) ++xi;", COD_PINS),
    "cod_expiry_strict": ("cod.c", "c->sn[c->head].t + c->N <= i", "c->sn[c->head].t + c->N < i", COD_PINS),
    "cod_b_not_downdated": ("cod.c", "for (int b = 0; b < dy; ++b) br[b] -= bh[e] * sn.H[(int64_t)b * xi + e];",
                            "for (int b = 0; b < dy; ++b) br[b] -= 0.0 * bh[e] * sn.H[(int64_t)b * xi + e];",
                            COD_PINS),
    "cod_restore_sign": ("cod.c", "MW[(int64_t)a * dy + b] += acc - sub;", "MW[(int64_t)a * dy + b] += acc + sub;",
                         COD_PINS),
    "power_iteration_step": ("fd.c", "for (int it = 0; it < steps; ++it) {", "for (int it = 1; it < steps; ++it) {",
                             FD_PINS + WINDOW_PINS),
}


def _build_mutant(tmp, name):
    fname, old, new, pins = MUTANTS[name]
    src = os.path.join(tmp, "src")
    shutil.copytree(ORACLE, src, ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    path = os.path.join(src, fname)
    text = open(path).read()
    assert text.count(old) >= 1, f"{name}: pattern not found in {fname}"
    open(path, "w").write(text.replace(old, new))
    sys.path.insert(0, ROOT)
    from oracle import build as ob
    return ob.build(src_dir=src, out=os.path.join(tmp, "liboracle_mutant.so")), pins


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    lib, pins = _build_mutant(str(tmp_path), name)
    env = dict(os.environ, SKETCH_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"]
                       + pins, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
