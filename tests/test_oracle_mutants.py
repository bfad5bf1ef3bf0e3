"""Plausible mistakes planted in a copy of the oracle must fail its pins.

Each mutant is the oracle source with one textual change (a dropped round, an
unstable output or routing loop, an off-by-one sample or splitter index, a
reversed tie-break, a strict/non-strict comparison swapped, a sample left
unordered by position).  The copy is compiled into
a temporary library and the pins of ``test_oracle.py`` are run against it in a
child process: at least one must fail (a crash of the child counts as caught).
"""
import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
import tests.test_oracle as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "sr4.c")

MUTANTS = {
    "output_loop_backward": (
        "    for (size_t i = 0; i < n; ++i) {                       /* output pass, forward */",
        "    for (size_t i = n; i-- > 0;) {                         /* output pass, forward */"),
    "last_round_dropped": (
        "    for (int lo = begin_bit; lo < end_bit; lo += digit_bits) {\n"
        "        int width = end_bit - lo < digit_bits ? end_bit - lo : digit_bits;\n"
        "        round_u32(",
        "    for (int lo = begin_bit; lo + digit_bits < end_bit; lo += digit_bits) {\n"
        "        int width = end_bit - lo < digit_bits ? end_bit - lo : digit_bits;\n"
        "        round_u32("),
    "splitter_index_off_by_one": (
        "        split_key[i - 1] = Sk[i * s - 1];\n        split_g[i - 1] = Sg[i * s - 1];",
        "        split_key[i - 1] = Sk[i * s];\n        split_g[i - 1] = Sg[i * s];"),
    "sample_segment_start_not_end": (
        "uint64_t q = (j * Nk + s - 1) / s - 1;",
        "uint64_t q = ((j - 1) * Nk + s - 1) / s;"),
    "composite_ties_reversed": (
        "return ka < kb || (ka == kb && ga < gb);",
        "return ka < kb || (ka == kb && ga > gb);"),
    "merge_ties_reversed": (
        "return a.key < b.key || (a.key == b.key && a.run < b.run);",
        "return a.key < b.key || (a.key == b.key && a.run > b.run);"),
    "ger_sample_not_ordered_by_position": (
        "rc = lsd_u32(Tg, Tk, m, 8, 0, 32, Ug, Uk);        /* by position */",
        "memcpy(Ug, Tg, m * 4); memcpy(Uk, Tk, m * 4);"),
    "gvr_sample_not_ordered_by_position": (
        "rc = lsd_u32(Tg, Tk, m, 8, 0, 32, Ug, Uk);        /* by input position */",
        "memcpy(Ug, Tg, m * 4); memcpy(Uk, Tk, m * 4);"),
    "gvr_bucket_search_nonstrict": (
        "if (comp_less(split_key[mid], split_g[mid], keys_in[q], q))",
        "if (!comp_less(keys_in[q], q, split_key[mid], split_g[mid]))"),
    "gvr_route_backward": (
        "    for (size_t q = 0; q < n; ++q) {\n        uint64_t o = start[bucket[q]]++;",
        "    for (size_t q = n; q-- > 0;) {\n        uint64_t o = start[bucket[q]]++;"),
    "float_negatives_not_reversed": (
        "    return a < b ? 1 : -1;                            /* float, both negative: reversed */",
        "    return a < b ? -1 : 1;                            /* float, both negative: reversed */"),
    "merge_ties_take_right": (
        "if (cmp_kind(k[j], k[i], bits, kind) < 0) { tk[o] = k[j]; tv[o++] = v[j++]; }",
        "if (cmp_kind(k[j], k[i], bits, kind) <= 0) { tk[o] = k[j]; tv[o++] = v[j++]; }"),
    "split_strict_instead_of_nonstrict": (
        "if (!comp_less(split_key[i - 1], split_g[i - 1], X[lo[k] + mid], lo[k] + mid))",
        "if (comp_less(X[lo[k] + mid], lo[k] + mid, split_key[i - 1], split_g[i - 1]))"),
}

PINS = [
    pins.test_exhaustive_small_alphabet_vs_insertion_sort,
    lambda: pins.test_random_vs_python_sorted(8),
    pins.test_large_vs_numpy_stable_argsort,
    pins.test_round_invariant_after_each_round,
    pins.test_special_cases_closed_form,
    lambda: pins.test_gsd_output_bounds_and_split("zipf"),
    pins.test_gsd_ragged_and_small,
    pins.test_gsd_closed_form_identity_input,
    pins.test_gsd_splitters_brute_force,
    lambda: pins.test_ger_output_split_and_splitters("zipf"),
    lambda: pins.test_ger_output_split_and_splitters("equal"),
    lambda: pins.test_gvr_output_split_and_splitters("zipf"),
    lambda: pins.test_gvr_output_split_and_splitters("equal"),
    pins.test_gvr_small_and_degenerate,
    lambda: pins.test_signed_vs_numpy(np.int32),
    lambda: pins.test_float_vs_numpy(np.float32),
    pins.test_float_total_order_special_values,
]


def _pins_pass():
    for pin in PINS:
        try:
            pin()
        except (AssertionError, ValueError):
            return False
    return True


def _run_mutant(so_path):
    """Child process: load the mutant library in place of the oracle, run the
    pins; exit 0 if they all pass (the mutant survived), 1 otherwise."""
    oracle._lib = oracle._configure(ctypes.CDLL(so_path))
    sys.exit(0 if _pins_pass() else 1)


def _child_verdict(source_text, tmp_path):
    c = tmp_path / "mutant.c"
    so = tmp_path / "libmutant.so"
    c.write_text(source_text)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", str(so), str(c)])
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = "import tests.test_oracle_mutants as m; m._run_mutant(%r)" % str(so)
    return subprocess.call([sys.executable, "-c", code], cwd=root,
                           stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL, timeout=600)


def test_control_copy_survives(tmp_path):
    """The harness itself: an unmodified copy run the same way passes every pin."""
    assert _child_verdict(open(SRC).read(), tmp_path) == 0


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_fails_some_pin(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, "mutation anchor missing: " + name
    rc = _child_verdict(src.replace(old, new, 1), tmp_path)
    assert rc != 0, "mutant %s survived every pin" % name


def test_unmutated_oracle_passes_all_pins():
    assert _pins_pass()
