"""Each plausible mistake planted in a copy of the oracle's C source must be
caught by at least one pin (no GPU).  The real oracle is never modified."""
import os
import tempfile

import pytest

from oracle import build as B
from oracle import oracle as O

from oracle_pins import ALL_PINS

MUTANTS = {
    "drop_self_loop_term": ("y[i * c + q] = acc + delta[i] * x[i * c + q];",
                            "y[i * c + q] = acc;"),
    "row_scale_twice": ("a[p] = (g->w[p] * s[i]) * s[g->col[p]];",
                        "a[p] = (g->w[p] * s[i]) * s[i];"),
    "weight_one_over_m": ("return 1.0 / (double)(m - 1);", "return 1.0 / (double)m;"),
    "degree_without_sigma": ("double ti = g->deg[i] + sigma;", "double ti = g->deg[i];"),
    "no_sqrt": ("1.0 / sqrt(ti)", "1.0 / ti"),
    "combine_ignores_alpha": ("acc = acc + alpha[t] * saved", "acc = acc + saved"),
    "no_dedupe": ("if (m == 0 || dst[i] != dst[m - 1]) dst[m++] = dst[i];",
                  "dst[m++] = dst[i];"),
    "merge_keeps_last": ("g->w[q] = g->w[q] + t[i].w;", "g->w[q] = t[i].w;"),
    "star_weight_as_clique": ("return (double)m / (double)(m - 1);",
                              "return 1.0 / (double)(m - 1);"),
    "virtual_mean_off_by_one": ("sum / (double)(hi - lo)", "sum / (double)(hi - lo + 1)"),
    "self_loop_unscaled": ("delta[i] = (sigma * s[i]) * s[i];", "delta[i] = sigma * s[i];"),
    "fixed_rows_not_restored": ("(fixed && fixed[i]) ? x_in[i * c + q] : acc", "acc"),
    "wirelength_unweighted": ("s = s + w * (d * d);", "s = s + (d * d);"),
    "hpwl_min_not_tracked": ("if (ga < mn) mn = ga;", "if (ga < mn) mx = ga;"),
    "exact_filter_without_identity": ("q[i] = 2.0 * p[i] - acc;", "q[i] = p[i] - acc;"),
    "cg_beta_inverted": ("double beta = rho_new / rho;", "double beta = rho / rho_new;"),
    "import_degree_skips_first": ("  for (int64_t r = 0; r < num_rows; ++r) {\n    double d = 0.0;\n    for (int64_t p = g->row_ptr[r]; p",
                                  "  for (int64_t r = 0; r < num_rows; ++r) {\n    double d = 0.0;\n    for (int64_t p = g->row_ptr[r] + 1; p"),
    "import_accepts_diagonal": ("col[p] >= num_rows || col[p] == r)", "col[p] >= num_rows)"),
    "star_order_lower_median": ("? g->ucell[a + m / 2] : 0", "? g->ucell[a + (m - 1) / 2] : 0"),
    "star_order_labels_ignore_rank": ("int32_t vid = (int32_t)(num_cells + vrank[e]);",
                                      "int32_t vid = (int32_t)(num_cells + vrank[e] / 2);"),
    "overflow_counts_deficits": ("if (e > 0.0) s = s + e;", "s = s + e;"),
    "overflow_bin_area_unsquared": ("double area = ((xh - xl) / (double)nbx) * ((yh - yl) / (double)nby);",
                                    "double area = (xh - xl) / (double)nbx;"),
    "density_overlap_not_clipped": ("double lx = (x1 < a1 ? x1 : a1) - (x0 > a0 ? x0 : a0);",
                                    "double lx = x1 - (x0 > a0 ? x0 : a0);"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    old, new = MUTANTS[name]
    src = open(B.SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "mutant.c")
        with open(path, "w") as f:
            f.write(src.replace(old, new))
        lib = O.load(B.build(os.path.join(d, "libmutant.so"), path))
        caught = []
        for pin in ALL_PINS:
            try:
                pin(lib)
            except Exception as exc:  # any failed pin counts
                caught.append((pin.__name__, type(exc).__name__))
        assert caught, f"no pin catches mutant {name}"
