"""Audit of the oracle's pins: every plausible mistake planted in a copy of the
oracle (on the CPU) must make at least one pin fail."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "orc.c")

# (name, original text, planted mistake)
MUTATIONS = [
    ("field_update_sign", "he[c->ci[e]] -= two_s * c->cj[e];", "he[c->ci[e]] += two_s * c->cj[e];"),
    ("field_uses_new_spin", "int32_t two_s = 2 * s[i]; /* the old spin value */",
     "int32_t two_s = -2 * s[i];"),
    ("accept_off_by_one", "if (d <= 0) {", "if (d <= 1) {"),
    ("dropped_factor_two", "exp(-2.0 * beta * (double)d)", "exp(-beta * (double)d)"),
    ("energy_step", "c->E[w] += 2 * d;", "c->E[w] += d;"),
    ("uniform_scale", "double uniform = (double)u * 0x1p-32; /* in [0, 1) */",
     "double uniform = (double)u * 0x1p-31;"),
    ("reverse_order", "for (int32_t i = 0; i < N; i++) {\n    uint32_t u = orc_mt_next(g);",
     "for (int32_t i = N - 1; i >= 0; i--) {\n    uint32_t u = orc_mt_next(g);"),
    ("swap_delta_sign", "(c->beta[k] - c->beta[k + 1]) * (double)(c->E[a] - c->E[b])",
     "(c->beta[k + 1] - c->beta[k]) * (double)(c->E[a] - c->E[b])"),
    ("swap_label", "c->temp_of[a] = k + 1;", "c->temp_of[a] = k;"),
    ("swap_parity", "orc_swap_round(c, (int32_t)(c->rounds & 1));", "orc_swap_round(c, 0);"),
    ("swap_skips_draw", "uint32_t u = orc_mt_next(&c->swap);",
     "uint32_t u = delta < 0.0 ? orc_mt_next(&c->swap) : 0u;"),
    ("mt_temper_const", "0x9d2c5680u", "0x9d2c5780u"),
    ("mt_temper_shift", "w ^= w >> 11;", "w ^= w >> 12;"),
    ("mt_twist_offset", "g->x[(k + 397) % 624]", "g->x[(k + 396) % 624]"),
    ("mt_seed_mult", "1812433253u", "1812433257u"),
    ("energy_field_sign", "e -= (int64_t)c->h[i] * s[i];", "e += (int64_t)c->h[i] * s[i];"),
    ("init_bit", "(orc_mt_next(&c->mt[w]) >> 31) ? 1 : -1", "(orc_mt_next(&c->mt[w]) & 1u) ? 1 : -1"),
    ("near_width_narrow", "fabs(uniform - p) < 1e-12) c->sw_near[k]++;", "fabs(uniform - p) < 1e-15) c->sw_near[k]++;"),
    ("near_width_wide", "fabs(uniform - p) < 1e-12) c->sw_near[k]++;", "fabs(uniform - p) < 1e-11) c->sw_near[k]++;"),
    ("near_wrong_pair", "fabs(uniform - p) < 1e-12) c->sw_near[k]++;", "fabs(uniform - p) < 1e-12) c->sw_near[k + 1]++;"),
    ("near_only_rejected", "if (delta < 0.0 && fabs(uniform - p) < 1e-12)", "if (delta < 0.0 && !accept && fabs(uniform - p) < 1e-12)"),
    ("swap_accept_le", "int accept = (delta >= 0.0) || (uniform < p);", "int accept = (delta >= 0.0) || (uniform <= p + 1e-13);"),
]

RUNNER = r"""
import sys
from tests import pins_oracle as p
for pin in p.ALL_PINS:
    try:
        pin()
    except Exception as e:
        print("CAUGHT_BY", pin.__name__, type(e).__name__)
        sys.exit(3)
print("NOT_CAUGHT")
"""


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(name, old, new, tmp_path):
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
