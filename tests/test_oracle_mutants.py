"""Plant plausible mistakes in copies of the oracle (on the CPU) and check
that each one fails at least one pin of tests/oracle_pins.py.

A mutant is a one-edit copy of oracle/esi_oracle.c: a flipped sign, a
dropped term, a wrong index, a swapped operand or an off-by-one in a
comparison.  It is compiled into a temporary directory and loaded in place
of the real oracle; the real oracle is never modified.
"""
import os
import subprocess
import sys

import pytest

import oracle

SRC = os.path.join(os.path.dirname(oracle.__file__), "esi_oracle.c")

# (name, text in the oracle, replacement)
MUTANTS = [
    ("add_sign", "S[q] = (S[q] + pol * C) * d;", "S[q] = (S[q] - pol * C) * d;"),
    ("decay_dropped", "S[q] = (S[q] + pol * C) * d;", "S[q] = (S[q] + pol * C);"),
    ("decay_then_add_in_default", "S[q] = (S[q] + pol * C) * d;", "S[q] = S[q] * d + pol * C;"),
    ("u_sign", "double u = 1.0 - k * dt;", "double u = 1.0 + k * dt;"),
    ("pow_operand_swap", "return pow(u, b);", "return pow(b, u);"),
    ("pow_as_product", "return pow(u, b);", "return u * b;"),
    ("dt_reversed", "int64_t dt = t[i] - T[q];", "int64_t dt = T[q] - t[i];"),
    ("T_not_updated", "T[q] = t[i];\n", "\n"),
    ("clamp_max_dropped", "    if (s > s_max)\n        s = s_max;\n", "\n"),
    ("clamp_min_dropped", "    if (s < s_min)\n        s = s_min;\n", "\n"),
    ("clamp_before_update", "        S[q] = clamp_s(S[q], s_min, s_max);\n        N[q] += 1;",
     "        N[q] += 1;"),
    # the clamp ahead of the add and decay instead of after them
    ("clamp_before_add",
     "            S[q] = (S[q] + pol * C) * d;\n        T[q] = t[i];\n        S[q] = clamp_s(S[q], s_min, s_max);\n",
     "            S[q] = (clamp_s(S[q], s_min, s_max) + pol * C) * d;\n        T[q] = t[i];\n"),
    ("frame_membership_off_by_one", "while (j < nf && t_frames[j] < t[i])",
     "while (j < nf && t_frames[j] <= t[i])"),
    ("map_denominator", "return (v - s_min) / (s_max - s_min);", "return (v - s_min) / (s_max + 1.0);"),
    ("map_offset", "return (v - s_min) / (s_max - s_min);", "return (v - s_max) / (s_max - s_min);"),
    ("pixel_index_transposed", "const int64_t q = (int64_t)y[i] * W + x[i];",
     "const int64_t q = (int64_t)x[i] * H + y[i];"),
    ("polarity_count", "P[q] += pol;", "P[q] += 1;"),
    ("negative_dt_kept", "        if (dt < 0)\n            dt = 0;\n        const double d",
     "        const double d"),
    ("snapshot_not_decayed", "v = clamp_s(S * decay_of((double)dt, k, b, flags), s_min, s_max);",
     "v = clamp_s(S, s_min, s_max);"),
    ("snapshot_decay_from_zero", "int64_t dt = t_f - T;", "int64_t dt = t_f;"),
    ("out_of_range_x_only", "if (x[i] >= W || y[i] >= H) {", "if (x[i] >= W) {"),
    ("unsorted_flag_dropped", "*unsorted = 1;", "(void)0;"),
    ("init_T_zero", "T[q] = t0;", "T[q] = 0;"),
    ("u8_round_down", "volatile float a = m + 0.5f;", "volatile float a = m;"),
    ("decay_then_add_order", "S[q] = S[q] * d + pol * C;", "S[q] = (S[q] + pol * C) * d;"),
    ("lazy_ignored", "if (!(flags & ORACLE_SNAPSHOT_LAZY)) {", "if (1) {"),
    ("exp_sign", "return exp(-k * dt);", "return exp(k * dt);"),
    ("exp_k_dropped", "return exp(-k * dt);", "return exp(-dt);"),
    ("exp_first_order", "return exp(-k * dt);", "return 1.0 - k * dt;"),
    ("exp_flag_ignored", "    if (flags & ORACLE_DECAY_EXP)\n        return esi_oracle_decay_exp(dt, k);\n", ""),
]


def _compile(tmp_path, name, old, new):
    """Write and build the mutant; returns the library path."""
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutant {name}: pattern must occur exactly once"
    path = tmp_path / f"m_{name}.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / f"libm_{name}.so"
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                    "-w", "-o", str(lib), str(path), "-lm"], check=True)
    return str(lib)


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new):
    # Each mutant runs in its own process: a mutant that writes out of
    # bounds may crash, which counts as caught.
    lib = _compile(tmp_path, name, old, new)
    here = os.path.dirname(os.path.abspath(__file__))
    env = dict(os.environ, PYTHONPATH=os.pathsep.join([here, os.path.dirname(here)]))
    r = subprocess.run([sys.executable, os.path.join(here, "oracle_pins.py"), lib],
                       capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode != 0, f"mutant {name} passes every pin: {r.stdout}"
