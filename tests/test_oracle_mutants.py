"""The pins must catch plausible mistakes in the oracle.

Each case plants one mistake in a temporary copy of the oracle's C source
(a wrong sign, a dropped term, a flipped tie-break or heuristic, an
off-by-one), builds it, and runs the pin tests against that build in a
subprocess: they must fail.  Nothing here touches the real oracle build.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "louvain_oracle.c")

MUTANTS = {
    "score_sign": ("- (i128)delta[i] * (i128)degc[cand]", "+ (i128)delta[i] * (i128)degc[cand]"),
    "own_deg_keeps_i": ("(i128)(degc[ci] - delta[i])", "(i128)(degc[ci])"),
    "tie_to_max_label": ("(s == s_best && cand < best)", "(s == s_best && cand > best)"),
    "singlet_direction": ("size[best] == 1 && best > ci", "size[best] == 1 && best < ci"),
    "move_on_equal_gain": ("if (best >= 0 && s_best > s_own)", "if (best >= 0 && s_best >= s_own)"),
    "loop_in_move_score": ("if (j == i) { loop += w[e]; continue; }", "if (j == i) { loop += w[e]; }"),
    "modularity_drops_loops": ("if (c[col[e]] == c[i])\n", "if (c[col[e]] == c[i] && col[e] != i)\n"),
    "accept_non_strict": ("(lh == rh && ll > rl)", "(lh == rh && ll >= rl)"),
    "contract_unmapped_row": ("int32_t b = newc[col[e]];", "int32_t b = newc[i];"),
    "renumber_off_by_one": ("map[v] = present ? (int32_t)k : -1;", "map[v] = present ? (int32_t)(k > 0 ? k - 1 : 0) : -1;"),
    "merge_non_alone": ("        if (size[ci] != 1)\n            continue;\n        int32_t target = -1;",
                        "        if (size[ci] < 1)\n            continue;\n        int32_t target = -1;"),
    "merge_on_equal_gain": ("        if (s <= s_own)\n            continue;", "        if (s < s_own)\n            continue;"),
    "merge_two_communities": ("            else if (c[j] != target)\n                single = 0;",
                              "            else if (c[j] != target)\n                single = 1;"),
    "merge_singlet_direction": ("size[target] == 1 && target > ci", "size[target] == 1 && target < ci"),
    "merge_keeps_old_q": ("            community_state(ln, c, delta, degc, size);\n            q_prev = modularity_int(ln, rp, cl, wt, c, delta, tw, qscratch);\n",
                          "            community_state(ln, c, delta, degc, size);\n"),
    "degree_skips_first": ("for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)\n            s += w[e];",
                           "for (int64_t e = row_ptr[i] + 1; e < row_ptr[i + 1]; ++e)\n            s += w[e];"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mutated = src.replace(old, new)
    c_path = tmp_path / "mut.c"
    so_path = tmp_path / "libmut.so"
    c_path.write_text(mutated)
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-shared", "-fPIC", "-o", str(so_path), str(c_path)])
    env = dict(os.environ, LOUVAIN_ORACLE_LIB=str(so_path))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"pins did not catch mutant {name}:\n{r.stdout[-2000:]}"
