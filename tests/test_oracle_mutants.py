"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check
that the pins catch every one of them."""
import os
import subprocess

import pytest

import oracle
import test_oracle_pins as pins
import test_oracle_xcor as xpins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

# (name, original text, mutated text): each must occur exactly once
MUTANTS = [
    ("conj_dropped", "cim += lam[l] * (ai * br - ar * bi);", "cim += lam[l] * (ai * br + ar * bi);"),
    ("csd_swapped_orientation", "cim += lam[l] * (ai * br - ar * bi);", "cim += lam[l] * (ar * bi - ai * br);"),
    ("re_part_term_dropped", "cre += lam[l] * (ar * br + ai * bi);", "cre += lam[l] * (ar * br);"),
    ("psd_wrong_node", "pwb += lam[l] * (br * br + bi * bi);", "pwb += lam[l] * (ar * ar + ai * ai);"),
    ("twiddle_sign", "*s = -sin(th);", "*s = sin(th);"),
    ("twiddle_index", "twiddle((int64_t)bins[b] * n, F,", "twiddle((int64_t)bins[b] * (n + 1), F,"),
    ("taper_not_applied", "double v = w[n] * xi[n];", "double v = xi[n];"),
    ("uspli_sign", "met[5] = (Kd * pli * pli - 1.0) / (Kd - 1.0);", "met[5] = (Kd * pli * pli + 1.0) / (Kd - 1.0);"),
    ("dswpli_literal_square", "met[6] = dd != 0.0 ? (Sim * Sim - Q) / dd : 0.0;",
     "met[6] = A > 0.0 ? (Sim * Sim) / (A * A) : 0.0;"),
    ("plv_not_unit", "Ure += cre / mag;", "Ure += cre;"),
    ("pli_no_abs", "double pli = K > 0 ? fabs((double)G) / Kd : 0.0;", "double pli = K > 0 ? ((double)G) / Kd : 0.0;"),
    ("wpli_abs_missing", "A += fabs(cim);", "A += cim;"),
    ("band_not_mean", "band[p * NMET + m] = bandacc[m] / (double)B;", "band[p * NMET + m] = bandacc[m];"),
    ("cor_no_centering", "double da = a[n] - ma, db = b[n] - mb;", "double da = a[n], db = b[n];"),
    ("cor_sum_not_mean", "cor[p] = K > 0 ? acc / (double)K : 0.0;", "cor[p] = acc;"),
    ("taper_weight_ignored", "cre += lam[l] * (ar * br + ai * bi);", "cre += (ar * br + ai * bi);"),
    ("xcor_one_direction", "for (int64_t s = -L; s <= L; ++s) {", "for (int64_t s = 0; s <= L; ++s) {"),
    ("xcor_full_energy_of_advanced", "const double d = sqrt(eu * ev);", "const double d = sqrt((s >= 0 ? ea : eb) * ev);"),
    ("xcor_no_centering", "xa[n] = a[n] - ma;", "xa[n] = a[n];"),
    ("xcor_sum_not_mean", "out[p] = K > 0 ? acc / (double)K : 0.0;", "out[p] = acc;"),
    ("xcor_min_not_max", "if (r > best) {", "if (-r > -best) {"),
]

CHECKS = [
    lambda: pins.test_brute_force_tiny(16, "hann"),
    lambda: pins.test_brute_force_tiny(32, "dpss"),
    pins.test_spectra_match_rfft,
    lambda: pins.test_two_sinusoids_constant_lag(12.0),
    pins.test_rank1_zero_lag_exact,
    pins.test_cor_matches_corrcoef,
    pins.test_swap_is_hermitian,
    lambda: xpins.test_literal_formula(10, 9, 0),
    xpins.test_closed_forms,
    xpins.test_zero_lag_is_cor_and_invariants,
]


@pytest.mark.parametrize("name,orig,mut", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(tmp_path, name, orig, mut):
    src = open(SRC).read()
    assert src.count(orig) == 1, name
    bad = tmp_path / f"{name}.c"
    bad.write_text(src.replace(orig, mut))
    so = tmp_path / f"lib{name}.so"
    subprocess.run(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                    str(bad), "-o", str(so), "-lm"], check=True)
    caught = []
    with oracle.use_library(str(so)):
        for chk in CHECKS:
            try:
                chk()
            except AssertionError:
                caught.append(chk)
    assert caught, f"mutant {name} passed every pin"
