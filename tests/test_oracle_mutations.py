"""Planted mistakes in the oracle must be caught by its pins.

Each case rebuilds oracle.c with one plausible mistake (a dropped term, a
wrong index, an unstable walk, a transposed place order) and runs the pin
module against it in a fresh process; the pins must fail. Nothing here runs on
a GPU.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = {
    "exclusive_becomes_inclusive": (
        "off[(size_t)j * r + v] = running;\n            running += hist[(size_t)j * r + v];",
        "running += hist[(size_t)j * r + v];\n            off[(size_t)j * r + v] = running;"),
    "binning_walks_backwards": (
        "    for (size_t i = 0; i < n; i++) {\n        uint64_t k = load_key(src_keys, key_bits, i);\n        uint64_t v = digit_at(k, lo, width);",
        "    for (size_t i = n; i-- > 0;) {\n        uint64_t k = load_key(src_keys, key_bits, i);\n        uint64_t v = digit_at(k, lo, width);"),
    "place_ignores_begin_bit": ("    *lo = a;", "    *lo = j * d;"),
    "last_place_not_clipped": ("    if (b > end_bit) b = end_bit;\n", "\n"),
    "histogram_single_place": (
        "hist[(size_t)j * r + digit_at(k, lo, width)] += 1;",
        "hist[digit_at(k, lo, width)] += 1;"),
    "msd_place_order": (
        "    for (int j = 0; j < p; j++) {\n        int lo, width;\n        place_bits(begin_bit, end_bit, d, j, &lo, &width);\n        /*",
        "    for (int j = p - 1; j >= 0; j--) {\n        int lo, width;\n        place_bits(begin_bit, end_bit, d, j, &lo, &width);\n        /*"),
    "scan_off_by_one": (
        "        running += in[i];\n        out[i] = running;",
        "        out[i] = running;\n        running += in[i];"),
    "status_shift_31": ("return (status << 30) | (value & 0x3FFFFFFFu);",
                        "return (status << 31) | (value & 0x3FFFFFFFu);"),
    "values_left_behind": ("if (src_vals) dst_vals[dst] = src_vals[i];",
                           "if (src_vals) dst_vals[i] = src_vals[i];"),
    "digit_mask_one_bit_short": ("return (key >> lo) & ((1ull << width) - 1ull);",
                                 "return (key >> lo) & ((1ull << width) - 2ull);"),
    "signed_sign_bit_kept": ("    if (key_type == 1) {\n        k ^= top;",
                             "    if (key_type == 1) {\n        k ^= 0;"),
    "negative_floats_flip_sign_only": ("        if (k & top) k = ~k & all;",
                                       "        if (k & top) k ^= top;"),
    "positive_floats_unflipped": ("        else k ^= top;", "        else k ^= 0;"),
    "descending_ignored": ("    if (descending) k = ~k & all;", "    if (descending) k = k & all;"),
    "typed_gather_keeps_input_order": (
        "store_key(keys_out, key_bits, i, load_key(keys_in, key_bits, idx_out[i]));",
        "store_key(keys_out, key_bits, i, load_key(keys_in, key_bits, i));"),
    "segments_typed_sorts_raw_bits": (
        "        rc = oracle_sort_typed((const char *)keys_in + a * kb, vals_in ? vals_in + a : NULL,\n"
        "                               (char *)keys_out + a * kb, vals_out ? vals_out + a : NULL,\n"
        "                               key_bits, len, begin_bit, end_bit, d, key_type, descending);",
        "        rc = oracle_sort((const char *)keys_in + a * kb, vals_in ? vals_in + a : NULL,\n"
        "                         (char *)keys_out + a * kb, vals_out ? vals_out + a : NULL,\n"
        "                         key_bits, len, begin_bit, end_bit, d, NULL);"),
    "segments_typed_values_not_offset": (
        "        rc = oracle_sort_typed((const char *)keys_in + a * kb, vals_in ? vals_in + a : NULL,",
        "        rc = oracle_sort_typed((const char *)keys_in + a * kb, vals_in ? vals_in : NULL,"),
    "segments_typed_direction_dropped": (
        "key_bits, len, begin_bit, end_bit, d, key_type, descending);",
        "key_bits, len, begin_bit, end_bit, d, key_type, 0);"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique/present"
    mutant = tmp_path / "oracle_mutant.c"
    mutant.write_text(src.replace(old, new))
    so = tmp_path / "liboracle_mutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", str(mutant), "-o", str(so)])
    env = dict(os.environ, ONESWEEP_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"pins did not catch mutant {name}:\n{r.stdout[-2000:]}"
