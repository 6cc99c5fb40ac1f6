"""Mutation check of the oracle's pins (CPU only).

Each mutant is a copy of oracle/msgpm_oracle.c with one plausible mistake
planted in it, built in a temporary directory.  The pins that cover that part
of the method run in a child process against the mutant (MSGPM_ORACLE_LIB
points the oracle's handle at it) and must fail; the same pins pass against an
unmodified copy built the same way."""
import os
import subprocess
import sys

import pytest

import oracle

pytestmark = pytest.mark.slow

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LEVELS = "tests/test_oracle_levels.py"
PINS = "tests/test_oracle_pins.py"

# (name, [(text, replacement), ...], test file, -k selection)
MUTANTS = [
    ("restricted pass without the plane candidate",
     [("          pm_try(S, dir, x, y, clampi((int)rx, 0, W - 1), clampi((int)ry, 0, H - 1), Hm, &b);",
       "          (void)rx;\n          (void)ry;")],
     LEVELS, "plane_candidate"),
    ("random search centred before the plane candidate",
     [("      /* plane candidate: where the region plane sends p */",
       "      const int cdx0 = b.tx - x, cdy0 = b.ty - y;\n      /* plane candidate: where the region plane sends p */"),
      ("      const int cdx = b.tx - x, cdy = b.ty - y;", "      const int cdx = cdx0, cdy = cdy0;")],
     LEVELS, "centred_after_plane"),
    ("restricted cost refresh under the identity",
     [("        Hm = region_H(S, S->hlabel[dir][p]);", "        Hm = IDENT;")],
     LEVELS, "incumbent_costed"),
    ("random-search stream not keyed by the pass's slot",
     [("rng_block(S, (uint64_t)p, (uint64_t)k, (uint64_t)iter, 2, dir, slot, 0, u);",
       "rng_block(S, (uint64_t)p, (uint64_t)k, (uint64_t)iter, 2, dir, 1, 0, u);")],
     LEVELS, "centred_after_plane"),
    ("restricted pass after level l keyed by slot l",
     [("    pm_pass(S, l + 1, 1);", "    pm_pass(S, l, 1);")],
     LEVELS, "documented_schedule"),
    ("RANSAC stream keyed by the level instead of level + 1",
     [("rng_block(S, (uint64_t)b, (uint64_t)h, 0, 3, dir, level + 1, stage, u);",
       "rng_block(S, (uint64_t)b, (uint64_t)h, 0, 3, dir, level, stage, u);")],
     LEVELS, "keyed_by_level"),
    ("RANSAC stream not keyed by the stage",
     [("rng_block(S, (uint64_t)b, (uint64_t)h, 0, 3, dir, level + 1, stage, u);",
       "rng_block(S, (uint64_t)b, (uint64_t)h, 0, 3, dir, level + 1, 1, u);")],
     LEVELS, "keyed_by_level"),
    ("Fisher-Yates draw over the whole list",
     [("          int rj = j + (int)orc_draw(u[j], (uint32_t)(n - j));",
       "          int rj = (int)orc_draw(u[j], (uint32_t)n);")],
     LEVELS, "keyed_by_level"),
    ("strict level priority ignored",
     [("(stage == 1 && !S->merge_strict) || (bw_ < 0)", "(stage == 1) || (bw_ < 0)")],
     LEVELS, "merge_across_levels or two_level_layered"),
    ("later levels never replace an assigned pixel",
     [("(stage == 1 && !S->merge_strict) || (bw_ < 0)", "(bw_ < 0)")],
     LEVELS, "merge_across_levels"),
    ("finer level wins exact ties",
     [("  if (I1[ORC_PI_LEVEL] != I2[ORC_PI_LEVEL]) return I1[ORC_PI_LEVEL] < I2[ORC_PI_LEVEL];",
       "  if (I1[ORC_PI_LEVEL] != I2[ORC_PI_LEVEL]) return I1[ORC_PI_LEVEL] > I2[ORC_PI_LEVEL];")],
     LEVELS, "merge_across_levels"),
    ("region plane reset where a level has none",
     [("      if (best >= 0) S->hlabel[dir][p] = best;", "      S->hlabel[dir][p] = best;")],
     LEVELS, "label_inherited"),
    ("NNF update rounds half to even",
     [("const double fx = fmin(fmax(floor(qx + 0.5), 0.0), (double)(W - 1));",
       "const double fx = fmin(fmax(nearbyint(qx), 0.0), (double)(W - 1));")],
     PINS, "nnf_update_rounds"),
]


def _build(tmp, text):
    src = os.path.join(tmp, "msgpm_oracle.c")
    with open(src, "w") as f:
        f.write(text)
    return oracle.compile_oracle(src, os.path.join(tmp, "libmsgpm_oracle.so"))


def _run_pins(lib, path, sel):
    env = dict(os.environ, MSGPM_ORACLE_LIB=lib, PYTHONDONTWRITEBYTECODE="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        path, "-k", sel], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout[-2000:]


def test_unmodified_copy_passes_every_selection(tmp_path):
    lib = _build(str(tmp_path), open(oracle.SRC).read())
    for path in sorted({m[2] for m in MUTANTS}):
        sel = " or ".join(sorted({m[3] for m in MUTANTS if m[2] == path}))
        rc, out = _run_pins(lib, path, sel)
        assert rc == 0, out


@pytest.mark.parametrize("name,edits,path,sel", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_fails_a_pin(name, edits, path, sel, tmp_path):
    text = open(oracle.SRC).read()
    for old, new in edits:
        assert text.count(old) == 1, (name, old)
        text = text.replace(old, new)
    lib = _build(str(tmp_path), text)
    rc, out = _run_pins(lib, path, sel)
    assert rc == 1 and "failed" in out, (name, rc, out)
