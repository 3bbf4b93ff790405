"""Planted mistakes in the oracle must be caught by its pins.

Each case copies oracle/tip_oracle.cpp, plants one plausible mistake (a dropped
term, a wrong sign or comparison, a missing cap), builds the copy in a
temporary directory and runs a compact version of the pins against it.  At
least one pin must fail for every mutant; the unmodified source must pass.
All of this runs on the CPU.
"""
from __future__ import annotations

import os
import subprocess
from math import comb

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2010_08695_amd import graphgen as gg

import _props

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "tip_oracle.cpp")

MUTANTS = {
    "count_self_pair": ("if (w > x) {", "if (w >= x) {"),
    "count_drop_far_end": ("            out[w] += b;\n", ""),
    "choose2_sign": ("return c * (c - 1) / 2;", "return c * (c + 1) / 2;"),
    "bup_no_cap": ("std::max(level, supp[w] - shared)", "(supp[w] - shared)"),
    "bup_linear_shared": ("const int64_t shared = choose2(co[w]);",
                          "const int64_t shared = co[w] > 1 ? co[w] : 0;"),
    "bup_largest_level_first": ("const int64_t level = queue.begin()->first;\n"
                                "        std::vector<int32_t> bag = std::move(queue.begin()->second);\n"
                                "        queue.erase(queue.begin());",
                                "const int64_t level = queue.rbegin()->first;\n"
                                "        std::vector<int32_t> bag = std::move(queue.rbegin()->second);\n"
                                "        queue.erase(std::prev(queue.end()));"),
    "bup_counts_self_wedge": ("if (w == x) continue;\n                    ++walked;",
                              "++walked;\n                    if (w == x) continue;"),
    "support_in_ignores_member": ("if (w != x && member[w]) {", "if (w != x) {"),
    "support_levels_ge_strict": ("if (theta[w] >= theta[x]) ge += f;", "if (theta[w] > theta[x]) ge += f;"),
    "support_levels_gt_loose": ("if (theta[w] > theta[x]) gt += f;", "if (theta[w] >= theta[x]) gt += f;"),
}


def _build(tmp_path, name, edit):
    src = open(SRC).read()
    if edit is not None:
        old, new = edit
        assert src.count(old) == 1, f"mutation site for {name} not unique/found"
        src = src.replace(old, new)
    cpp = tmp_path / f"{name}.cpp"
    so = tmp_path / f"lib{name}.so"
    cpp.write_text(src)
    wing = os.path.join(os.path.dirname(SRC), "wing_oracle.cpp")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", str(cpp), wing, "-o", str(so)])
    return oracle._load(str(so))


def _pins_pass(lib) -> bool:
    try:
        rng = np.random.default_rng(3)
        for i in range(25):
            g = gg.tiny_random(int(rng.integers(3, 9)), int(rng.integers(3, 8)),
                               float(rng.choice([0.4, 0.6, 0.8])), 9000 + i)
            bu, bv, tot = oracle.count(g, lib=lib)
            b = brute.butterflies(g)
            assert tot == b[2] and (bu == b[0]).all() and (bv == b[1]).all()
            for side in (0, 1):
                assert (oracle.bup(g, side, lib=lib)[0] == brute.tip_numbers(g, side)).all()
        for a, b_ in ((3, 4), (5, 2), (6, 6)):
            g = gg.complete_bipartite(a, b_)
            assert (oracle.bup(g, 0, lib=lib)[0] == (a - 1) * comb(b_, 2)).all()
        g = gg.config_graph("plain-small")
        _th, _order, wedges = oracle.bup(g, 0, lib=lib)
        dv = np.bincount(g.ev, minlength=g.n_v).astype(np.int64)
        assert wedges == int((dv * (dv - 1)).sum())
        g = gg.chung_lu(200, 80, 1500, 2.3, 2.1, seed=41)
        th = oracle.bup(g, 0, lib=lib)[0]
        member = (th >= np.unique(th)[len(np.unique(th)) // 2]).astype(np.uint8)
        h = np.nonzero(member)[0].astype(np.int32)
        f = oracle.support_in(g, 0, member, h, lib=lib)
        assert int(f.min()) == int(th[h].min())
        # tip numbers satisfy the certificate f_x(theta >= theta_x) >= theta_x
        # and, at x's peel, f_x(theta > theta_x) <= theta_x; counts match
        q = np.arange(g.n_u, dtype=np.int32)
        lv = oracle.support_levels(g, 0, th, q, lib=lib)
        assert (lv[:, 0] == oracle.count(g, lib=lib)[0]).all()
        assert (lv[:, 1] >= th).all() and (lv[:, 2] <= th).all()
        return True
    except AssertionError:
        return False


def test_unmodified_oracle_passes(tmp_path):
    assert _pins_pass(_build(tmp_path, "orig", None))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    assert not _pins_pass(_build(tmp_path, name, MUTANTS[name])), f"mutant {name} survived"
