"""Planted mistakes in the edge/wing/k-tip oracle (oracle/wing_oracle.cpp)
must be caught by its pins: each case builds a copy with one plausible
mistake (a dropped term, a missing cap, a skipped liveness check, a wrong
comparison) and runs a compact version of tests/test_oracle_wing_pins.py
against it.  The unmodified source must pass.  CPU only."""
from __future__ import annotations

import os
import subprocess

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2010_08695_amd import graphgen as gg

HERE = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(HERE, "oracle", "wing_oracle.cpp")
TIP_SRC = os.path.join(HERE, "oracle", "tip_oracle.cpp")

MUTANTS = {
    "edge_count_keeps_v": ("if (xu.first != u) s += co[xu.first] - 1;", "if (xu.first != u) s += co[xu.first];"),
    "edge_count_self_pair": ("if (xu.first != u) s += co[xu.first] - 1;", "s += co[xu.first] - 1;"),
    "wing_no_cap": ("std::max(level, supp[f] - 1)", "(supp[f] - 1)"),
    "wing_drops_far_edge": ("                    lower(e4);\n", ""),
    "wing_uses_removed_edge": ("if (u2 == u || gone[e3]) continue;", "if (u2 == u) continue;"),
    "wing_tags_removed_edges": ("if (!gone[yv.second]) tag[yv.first] = yv.second;", "tag[yv.first] = yv.second;"),
    "ktip_one_shared_neighbour": ("if (co[w] >= 2 && comp[w] < 0)", "if (co[w] >= 1 && comp[w] < 0)"),
    "ktip_strict_threshold": ("if (theta[s] < k || comp[s] >= 0) continue;", "if (theta[s] <= k || comp[s] >= 0) continue;"),
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
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", TIP_SRC, str(cpp), "-o", str(so)])
    return oracle._load(str(so))


def _pins_pass(lib) -> bool:
    try:
        rng = np.random.default_rng(4)
        n_wing = 0
        for i in range(80):
            g = gg.tiny_random(int(rng.integers(2, 7)), int(rng.integers(2, 6)), float(rng.choice([0.6, 0.8, 1.0])),
                               7000 + i)
            assert (oracle.edge_count(g, lib=lib) == brute.edge_butterflies(g)).all()
            if brute.canonical(g)[0].shape[0] <= 12:
                n_wing += 1
                assert (oracle.wing(g, lib=lib)[0] == brute.wing_numbers(g)).all()
            th = oracle.bup(g, 0, lib=lib)[0]
            for k in sorted(set(th.tolist()) | {1}):
                assert (oracle.ktip(g, 0, th, k, lib=lib) == brute.ktips(g, 0, k)).all()
        assert n_wing >= 20
        for a, b in ((3, 4), (4, 4), (2, 5)):
            g = gg.complete_bipartite(a, b)
            assert (oracle.wing(g, lib=lib)[0] == (a - 1) * (b - 1)).all()
        return True
    except AssertionError:
        return False


def test_unmodified_wing_oracle_passes(tmp_path):
    assert _pins_pass(_build(tmp_path, "orig", None))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_wing_mutant_is_caught(tmp_path, name):
    assert not _pins_pass(_build(tmp_path, name, MUTANTS[name])), f"mutant {name} survived"
