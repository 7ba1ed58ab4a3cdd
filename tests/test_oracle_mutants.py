"""Plant mistakes in a copy of the oracle (on the CPU) and require the pins to
catch every one of them.  A pin suite that passes a broken oracle would not
be pinning anything."""
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (name, text in cspd_oracle.c, replacement) -- each a plausible slip.
MUTANTS = [
    ("no_angle_normalisation", "double score = fabs(dot) / nu[c];", "double score = fabs(dot);"),
    ("tie_to_highest_index", "if (score > bs) { ss = bs;", "if (score >= bs) { ss = bs;"),
    ("residue_sign", "s -= asub[(size_t)j * M + i] * beta[j];", "s += asub[(size_t)j * M + i] * beta[j];"),
    ("interleaved_children", "cand[nc++] = sorted[i] * Q + q;", "cand[nc++] = q * md->atoms[s - 1] + sorted[i];"),
    ("back_substitution_transposed", "s -= w[(size_t)k * m + j] * beta[k];", "s -= w[(size_t)j * m + k] * beta[k];"),
    ("phi_transposed", "acc += phi[(size_t)i * N + j] * d[map_s[j]];", "acc += phi[(size_t)j * M + i] * d[map_s[j]];"),
    ("phase_ignored", "(size_t)(phase ? phase[b] : 0);", "(size_t)(phase ? 0 : 0);"),
    ("phase_shifted", "effective_dict(md, s, maps[s], NULL, md->phi ? md->phi + (size_t)p * M * N : NULL,",
     "effective_dict(md, s, maps[s], NULL, md->phi ? md->phi + (size_t)((p + 1) % P) * M * N : NULL,"),
    ("reselect_chosen", "if (chosen[c] || nu[c] == 0.0) continue;", "if (nu[c] == 0.0) continue;"),
    ("mask_ignored", "a[j] = (md->phi_kind == OR_PHI_MASK && !mask[j]) ? 0.0 : u;", "a[j] = u;"),
    ("no_dependence_stop", "if (rlast * rlast <= OR_DEP_TOL * nu[pick] * nu[pick]) break;", "if (0) break;"),
    ("coef_reversed", "for (int j = 0; j < n; ++j) io->coef[j] = beta[j];", "for (int j = 0; j < n; ++j) io->coef[j] = beta[n - 1 - j];"),
    ("xhat_wrong_atom", "xb[j] += Df[(size_t)sup[k] * N + j] * cf[k];", "xb[j] += Df[(size_t)k * N + j] * cf[k];"),
    ("map_not_composed", "maps[s][j] = md->up_map[s][maps[s + 1][j]];", "maps[s][j] = md->up_map[s][j % md->dim[s + 1]];"),
    ("no_restart_of_residue", "memcpy(r, y, sizeof(double) * (size_t)M);\n    int n = 0;", "if (nc < 0) memcpy(r, y, sizeof(double) * (size_t)M);\n    int n = 0;"),
    # the per-step trace and the forced prefix behind the near-tie rule
    ("picked_score_is_best", "picked_score = fabs(dot) / nu[pick];", "picked_score = bs;"),
    ("first_max_every_step", "if (it == 0) first_max = bs;", "first_max = bs;"),
    ("forced_ignores_chosen", "if (cand[c] == want && !chosen[c] && nu[c] != 0.0) pick = c;",
     "if (cand[c] == want && nu[c] != 0.0) pick = c;"),
    ("runner_up_not_tracked", "else if (score > ss) { ss = score; second = c; }", "else if (0) { ss = score; second = c; }"),
    ("forced_ignored", "if (io->forced && io->forced[it] >= 0) {", "if (io->forced && io->forced[it] >= 0 && 0) {"),
]

RUNNER = r"""
import sys
sys.path[:0] = [{root!r}, {tests!r}]
import oracle_pins as P
failed = []
for pin in P.ALL_PINS:
    try:
        pin({lib!r})
    except Exception as e:
        failed.append(pin.__name__)
print("FAILED:" + ",".join(failed))
"""


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new):
    src = open(os.path.join(ROOT, "oracle", "cspd_oracle.c")).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    tmp = tempfile.mkdtemp(prefix="oracle_mutant_")
    try:
        path = os.path.join(tmp, "m.c")
        open(path, "w").write(src.replace(old, new))
        lib = os.path.join(tmp, "libm.so")
        oracle.build(src=path, out=lib)
        code = RUNNER.format(root=ROOT, tests=os.path.join(ROOT, "tests"), lib=lib)
        p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
        # a crash of the mutant also counts as caught
        if p.returncode == 0:
            line = [l for l in p.stdout.splitlines() if l.startswith("FAILED:")][-1]
            assert line != "FAILED:", f"mutant {name} passed every pin"
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
