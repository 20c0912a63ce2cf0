"""CPU tests: the pins catch plausible mistakes planted in copies of the oracle.

Each case copies the oracle source into a temporary directory, plants one mistake by text
substitution, builds it, and checks that at least one pin fails. The oracle itself is never
modified.
"""
import os

import pytest

import oracle
import oracle_pins

MUTANTS = {
    "twiddle_sign": ("double wr = cos(ang), wi = sin(ang);", "double wr = cos(ang), wi = -sin(ang);"),
    "twiddle_angle": ("(double)k / (double)len", "(double)k / (double)h"),
    "mirror_not_conjugated": ("g[2 * c2 + 1] -= im;", "g[2 * c2 + 1] += im;"),
    "cell_transposed": ("size_t c1 = (size_t)mod_n(iv, N) * N + mod_n(iu, N);",
                        "size_t c1 = (size_t)mod_n(iu, N) * N + mod_n(iv, N);"),
    "round_half_up": ("double ru = nearbyint(xu);", "double ru = floor(xu + 0.5);"),
    "natural_weight_halved": ("W = 2.0 * (double)kept;", "W = (double)kept;"),
    "no_shift": ("const int s = shift ? N / 2 : 0;", "const int s = 0;"),
    "edge_not_strict": ("fabs(ru) < half && fabs(rv) < half", "fabs(ru) <= half && fabs(rv) <= half"),
    "cell_size_missing_dl": ("return cycles_per_metre * cells_per_wavelength;",
                             "return cycles_per_metre * (double)grid_n;"),
    "uniform_not_divided": ("g[2 * c] /= (double)cnt[c];\n                g[2 * c + 1] /= (double)cnt[c];",
                            "(void)g;"),
    "column_pass_drops_imag": ("col[2 * r + 1] = work[2 * ((size_t)r * N + c) + 1];",
                               "col[2 * r + 1] = 0.0;"),
    "image_transposed": ("image[(size_t)y * N + x] = w[0] * inv;", "image[(size_t)x * N + y] = w[0] * inv;"),
    "mirror_cell_wrong": ("size_t c2 = (size_t)mod_n(-iv, N) * N + mod_n(-iu, N);",
                          "size_t c2 = (size_t)mod_n(-iv, N) * N + mod_n(iu, N);"),
    "butterfly_sign": ("y[0] = x[0] - tr; y[1] = x[1] - ti;", "y[0] = x[0] + tr; y[1] = x[1] - ti;"),
    # direct transform
    "dft_phase_sign": ("img[(size_t)y * N + x] += 2.0 * (re * cos(phase) - im * sin(phase));",
                       "img[(size_t)y * N + x] += 2.0 * (re * cos(phase) + im * sin(phase));"),
    "dft_axes_swapped": ("const double phase = two_pi * (a * X + c * Y) / (double)N;",
                         "const double phase = two_pi * (a * Y + c * X) / (double)N;"),
    "dft_snap_ignored": ("const double a = snap ? ru : xu;", "const double a = xu;"),
    # convolutional gridding
    "conv_mirror_not_conjugated": ("spread(g, N, -xu, -xv, width, beta, re, -im);",
                                   "spread(g, N, -xu, -xv, width, beta, re, im);"),
    "conv_mirror_not_mirrored": ("spread(g, N, -xu, -xv, width, beta, re, -im);",
                                 "spread(g, N, -xu, xv, width, beta, re, -im);"),
    "conv_support_halved": ("const double h = 0.5 * width;", "const double h = 0.25 * width;"),
    "conv_kernel_no_sqrt": ("return exp(beta * (sqrt(1.0 - z * z) - 1.0));", "return exp(beta * ((1.0 - z * z) - 1.0));"),
    "conv_correction_not_centred": ("int X = shift ? x - N / 2 : (x < N / 2 ? x : x - N);",
                                    "int X = shift ? x : (x < N / 2 ? x : x - N);"),
    "conv_correction_one_axis": ("img[(size_t)y * N + x] /= corr[x] * corr[y];", "img[(size_t)y * N + x] /= corr[x] * corr[x];"),
    "conv_transform_frequency": ("cos(M_PI * nu * width * sin(t))", "cos(2.0 * M_PI * nu * width * sin(t))"),
    "conv_edge_not_strict": ("fabs(rv) < half && fabs(ru) < half", "fabs(rv) <= half && fabs(ru) <= half"),
    "conv_weight_halved": ("*weight_sum = 2.0 * (double)kept;", "*weight_sum = (double)kept;"),
    # visibility corrections
    "corr_rotation_sign": ("rot_im = sin(2.0 * M_PI * turns);", "rot_im = -sin(2.0 * M_PI * turns);"),
    "corr_w_term_dropped": ("x[2] * (n0 - 1.0)", "0.0 * x[2]"),
    "corr_w_term_not_relative": ("x[2] * (n0 - 1.0)", "x[2] * n0"),
    "corr_gain_conj_on_first": ("br = gj[0], bi = -(double)gj[1];", "br = gj[0], bi = (double)gj[1];"),
    "corr_antennas_swapped": ("ant_i[b] = i; ant_j[b] = j;", "ant_i[b] = j; ant_j[b] = i;"),
    "corr_frequency_missing": ("const double cycles_per_metre = freq_hz[c] / SPEED_OF_LIGHT;",
                               "const double cycles_per_metre = 150.0e6 / SPEED_OF_LIGHT;"),
    # correlation
    "cmac_conjugate_on_first": ("sim += (int64_t)xi[1] * xj[0] - (int64_t)xi[0] * xj[1];",
                                "sim += (int64_t)xi[0] * xj[1] - (int64_t)xi[1] * xj[0];"),
    "cmac_pol_products_swapped": ("if (P == 4) pp = 2 * p + q;", "if (P == 4) pp = p + 2 * q;"),
    "cmac_norm_missing_channels": ("const double count = (double)n_int * (double)n_favg;",
                                   "const double count = (double)n_int;"),
    "cmac_channel_groups_wrong": ("for (int f = c * n_favg; f < (c + 1) * n_favg; ++f)",
                                  "for (int f = c; f < c + n_favg; ++f)"),
    "cmac_baseline_order": ("const long b = (long)i * (i - 1) / 2 + j;", "const long b = (long)j * (j - 1) / 2 + i;"),
    # de-dispersion
    "dd_delay_sign": ("(1.0 / (f_mhz * f_mhz) - 1.0 / (ref_mhz * ref_mhz))",
                      "(1.0 / (ref_mhz * ref_mhz) - 1.0 / (f_mhz * f_mhz))"),
    "dd_delay_not_in_samples": ("nearbyint(delay_s / dt_s)", "nearbyint(delay_s)"),
    "dd_reference_lowest": ("if (freq_hz[c] > f_ref) f_ref = freq_hz[c];", "if (freq_hz[c] < f_ref) f_ref = freq_hz[c];"),
    "dd_no_shift": ("const int ts = t + delays[(size_t)k * C + c];", "const int ts = t;"),
    "dd_sum_not_mean": ("for (size_t i = 0; i < NN; ++i) o[i] /= (double)C;", "(void)C;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(tmp_path, name):
    before, after = MUTANTS[name]
    src = open(oracle.SRC).read()
    assert src.count(before) == 1, f"mutation site for {name} not found exactly once"
    path = tmp_path / "blink_ref_mutant.c"
    path.write_text(src.replace(before, after))
    lib = oracle.compile_library(str(path), str(tmp_path / f"libmut_{name}.so"))
    O = oracle.Oracle(oracle.load(lib))
    caught = []
    for pin in oracle_pins.PINS + oracle_pins.EXTRA_PINS:
        try:
            pin(O)
        except Exception:  # any failure of a pin counts as caught
            caught.append(pin.__name__)
    assert caught, f"no pin caught the planted mistake {name}"
    os.remove(lib)
