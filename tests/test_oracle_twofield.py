"""The oracle's two-field form against its pins (CPU only), and an audit: each
plausible mistake planted in a copy of the two-field code makes a pin fail."""
import os
import subprocess
import sys

import pytest

from . import pins_twofield

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "orc.c")


@pytest.mark.parametrize("pin", pins_twofield.TWO_FIELD_PINS, ids=lambda f: f.__name__)
def test_two_field_pin(pin):
    pin()


# (name, original text, planted mistake)
MUTATIONS = [
    ("tau_weight_is_a", "double x_t = cw * (double)d_t;", "double x_t = a * (double)d_t;"),
    ("field_switch_swapped", "int32_t *field = c->ctau[e] ? ht : hs;", "int32_t *field = c->ctau[e] ? hs : ht;"),
    ("bond_step_sign", "c->B[w] -= 2 * d_t;", "c->B[w] += 2 * d_t;"),
    ("swap_sign", "delta = d_sp - d_t;", "delta = d_sp + d_t;"),
    ("swap_space_energy", "int64_t esp_a = c->E[a] + c->B[a]", "int64_t esp_a = c->E[a] - c->B[a]"),
    ("dropped_factor_two", "accept = uniform < exp(-2.0 * x);", "accept = uniform < exp(-x);"),
    ("approx_arg", "orc_exp_approx((float)(-2.0 * x), kind)", "orc_exp_approx((float)(-x), kind)"),
    ("tau_into_space_field", "        ft += c->cj[e] * s[c->ci[e]];\n      else\n        f += c->cj[e] * s[c->ci[e]];\n    }\n    he[i] = f;",
     "        f += c->cj[e] * s[c->ci[e]];\n      else\n        f += c->cj[e] * s[c->ci[e]];\n    }\n    he[i] = f;"),
]

RUNNER = r"""
import sys
from tests import pins_twofield as p
for pin in p.TWO_FIELD_PINS:
    try:
        pin()
    except Exception as e:
        print("CAUGHT_BY", pin.__name__, type(e).__name__)
        sys.exit(3)
print("NOT_CAUGHT")
"""


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_two_field_mistake_is_caught(name, old, new, tmp_path):
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
