"""The oracle's pins catch plausible mistakes (CPU only).

Each case compiles a copy of oracle.c with one planted mistake into a
temporary directory, swaps it in for the real oracle and reruns the pin
checks of test_oracle.py; at least one pin must fail.  Only mistakes that
keep every memory access in bounds are planted.
"""
import os
import subprocess

import pytest

import oracle
from tests import test_oracle as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    # tie rule flipped: equal keys from B before those from A
    "merge_tie_strict": ("return ((const uint32_t *)A)[a] <= ((const uint32_t *)B)[b];",
                         "return ((const uint32_t *)A)[a] < ((const uint32_t *)B)[b];"),
    # float keys compared as raw bits
    "float_bits_compare": ("return ((const float *)A)[a] <= ((const float *)B)[b];",
                           "return ((const uint32_t *)A)[a] <= ((const uint32_t *)B)[b];"),
    # Algorithm 1: floor instead of ceiling when halving
    "alg1_floor_delta_j": ("(j - j_low + 1) / 2", "(j - j_low) / 2"),
    "alg1_floor_delta_k": ("(k - k_low + 1) / 2", "(k - k_low) / 2"),
    # Algorithm 1: wrong lower bound updated
    "alg1_klow_from_j": ("k_low = k;", "k_low = j;"),
    "alg1_jlow_from_k": ("j_low = j;", "j_low = k;"),
    # Algorithm 1: strict / non-strict tests swapped
    "alg1_cond2_strict": ("key_ge(kt, B, k - 1, A, j)", "key_gt(kt, B, k - 1, A, j)"),
    "alg1_cond1_nonstrict": ("key_gt(kt, A, j - 1, B, k)", "key_ge(kt, A, j - 1, B, k)"),
    # Algorithm 1: j_low started at 0 instead of max(0, i - n)
    "alg1_jlow_init": ("uint64_t j_low = i > n ? i - n : 0;", "uint64_t j_low = 0;"),
    # co-rank by definition returns k instead of j
    "brute_returns_k": ("    return a;\n}", "    return i - a;\n}"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path, monkeypatch, figure):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mutated = src.replace(old, new, 1)
    c_path = tmp_path / "oracle_mutant.c"
    so_path = tmp_path / "liboracle_mutant.so"
    c_path.write_text(mutated)
    subprocess.run(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", str(so_path),
                    str(c_path)], check=True)
    monkeypatch.setattr(oracle, "_lib", oracle.open_library(str(so_path)))
    failures = []
    checks = [lambda: c(figure) for c in pins.PIN_CHECKS[:4]]
    checks += [c for c in pins.PIN_CHECKS[4:]]
    checks += [lambda: pins.check_exhaustive(3, 4)]
    for check in checks:
        try:
            check()
        except (AssertionError, RuntimeError):
            failures.append(check)
    assert failures, f"no pin caught mutant {name}"
