"""The oracle's layer-pair order against its pins (CPU only), and an audit: each
plausible mistake planted in a copy of that code makes a pin fail."""
import os
import subprocess
import sys

import pytest

from . import pins_pairs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "orc.c")


@pytest.mark.parametrize("pin", pins_pairs.PAIR_PINS, ids=lambda f: f.__name__)
def test_pair_pin(pin):
    pin()


# (name, original text, planted mistake); the single-site step is shared with the
# canonical sweep and audited with it (test_oracle_mutations.py)
MUTATIONS = [
    ("odd_slices_first", "const int32_t m = 2 * t + parity;", "const int32_t m = 2 * t + 1 - parity;"),
    ("reverse_in_slice_order", "for (int32_t q = 0; q < S; q++) metropolis_at(c, w, m * S + q, orc_mt_next(g), beta);",
     "for (int32_t q = S - 1; q >= 0; q--) metropolis_at(c, w, m * S + q, orc_mt_next(g), beta);"),
    ("init_low_bit", "for (int32_t q = 0; q < S; q++) s[(2 * t + j) * S + q] = (orc_mt_next(g) >> 31) ? 1 : -1;",
     "for (int32_t q = 0; q < S; q++) s[(2 * t + j) * S + q] = (orc_mt_next(g) & 1u) ? 1 : -1;"),
    ("init_slices_swapped", "s[(2 * t + j) * S + q] = (orc_mt_next(g) >> 31)", "s[(2 * t + 1 - j) * S + q] = (orc_mt_next(g) >> 31)"),
    ("beta_of_walker", "const double beta = c->beta[c->temp_of[w]];\n  for (int32_t parity",
     "const double beta = c->beta[w];\n  for (int32_t parity"),
]

RUNNER = r"""
import sys
from tests import pins_pairs as p
for pin in p.PAIR_PINS:
    try:
        pin()
    except Exception as e:
        print("CAUGHT_BY", pin.__name__, type(e).__name__)
        sys.exit(3)
print("NOT_CAUGHT")
"""


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_pair_mistake_is_caught(name, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique/present: {name}"
    mut = tmp_path / "orc.c"
    mut.write_text(src.replace(old, new))
    hdr = os.path.join(ROOT, "oracle", "orc.h")
    so = tmp_path / "liboracle_mut.so"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11",
                    "-I", os.path.dirname(hdr), "-o", str(so), str(mut), "-lm", "-lpthread"], check=True)
    env = dict(os.environ, ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-c", RUNNER], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=300)
    assert "CAUGHT_BY" in r.stdout, f"{name}: no pin failed\n{r.stdout}\n{r.stderr[-2000:]}"
