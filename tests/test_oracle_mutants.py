"""Each plausible mistake planted in a copy of the oracle (on the CPU) must make
at least one pin fail -- evidence that the pins constrain the oracle."""
import os
import shutil
import tempfile

import pytest

import oracle
from tests import oracle_pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "tie_direction_flipped": ("if (tie == TIE_LOWER_KEEPS) return u < v;", "if (tie == TIE_LOWER_KEEPS) return u > v;"),
    "mex_starts_at_one": ("int32_t m = 0;\n    while (seen[m])", "int32_t m = 1;\n    while (seen[m])"),
    "recolour_reads_live_state": ("{ defective = 1; break; }\n            }\n            if (defective) {\n"
                                  "                colors[v] = smallest_free_colour(v, row_ptr, col_idx, snap, seen);",
                                  "{ defective = 1; break; }\n            }\n            if (defective) {\n"
                                  "                colors[v] = smallest_free_colour(v, row_ptr, col_idx, colors, seen);"),
    "detect_reads_live_state": ("loses(v, u, tie) && snap[u] == snap[v]) { defective = 1; break; }",
                                "loses(v, u, tie) && colors[u] == colors[v]) { defective = 1; break; }"),
    "round0_uncoloured": ("for (int32_t v = 0; v < n; ++v) colors[v] = 0;", "for (int32_t v = 0; v < n; ++v) colors[v] = -1;"),
    "seq_reverse_order": ("for (int32_t v = 0; v < n; ++v) colors[v] = smallest_free_colour(v, row_ptr, col_idx, colors, seen);",
                          "for (int32_t v = n - 1; v >= 0; --v) colors[v] = smallest_free_colour(v, row_ptr, col_idx, colors, seen);"),
    "worklist_not_swapped": ("int32_t *t = U; U = L; L = t; /* U^i <- L */", "/* U^i <- L forgotten */"),
    "check_ignores_degree_bound": ("if (colors[v] < 0 || colors[v] > d) ++bad;", "if (colors[v] < 0) ++bad;"),
    "mex_ignores_top_colour": ("if (cu >= 0 && cu <= d) seen[cu] = 1;", "if (cu >= 0 && cu < d - 1) seen[cu] = 1;"),
    "classes_counts_shifted": ("ptr[colors[v] + 1] += 1;", "ptr[colors[v]] += 1;"),
    "classes_descending_ids": ("for (int32_t v = 0; v < n; ++v) vtx[next[colors[v]]++] = v;",
                               "for (int32_t v = n - 1; v >= 0; --v) vtx[next[colors[v]]++] = v;"),
    "classes_range_unchecked": ("if (colors[v] < 0 || colors[v] >= K) return ORC_EINVAL;",
                                "if (colors[v] < 0) return ORC_EINVAL;"),
    "recolor_uncoloured_not_defective": ("int defective = snap[v] < 0 || snap[v] > d;", "int defective = 0;"),
    "recolor_touched_ignored": ("if (in_u0[v] || colors[v] < 0 || colors[v] > d) U[nU++] = v;",
                                "if (colors[v] < 0 || colors[v] > d) U[nU++] = v;"),
    "square_misses_two_hop": ("if (mark[w] != v) { mark[w] = v; row[len++] = w; }", "(void)w;"),
    "square_lists_self": ("mark[v] = v; /* v itself is never listed */", "/* v listed */"),
    "recolor_live_reads": ("if (u != v && loses(v, u, tie) && snap[u] == snap[v]) defective = 1;",
                           "if (u != v && loses(v, u, tie) && colors[u] == colors[v]) defective = 1;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, "mutation anchor not found: %s" % name
    d = tempfile.mkdtemp(prefix="orc_mut_")
    try:
        src = os.path.join(d, "oracle.c")
        with open(src, "w") as f:
            f.write(text.replace(old, new))
        lib = oracle.OracleLib(oracle.build(src=src, out=os.path.join(d, "liboracle.so")))
        failed = []
        for pin in oracle_pins.ALL_PINS:
            try:
                pin(lib)
            except (AssertionError, RuntimeError, IndexError, ValueError):
                failed.append(pin.__name__)
        assert failed, "no pin caught mutant %s" % name
    finally:
        shutil.rmtree(d, ignore_errors=True)
