"""The seeded input generators: determinism, sizes and shape of the draws."""
import numpy as np

from paper_2010_08695_amd import graphgen as gg


def test_plain_small_shape_and_determinism():
    a = gg.config_graph("plain-small")
    b = gg.config_graph("plain-small")
    assert (a.n_u, a.n_v, a.m) == (2000, 1000, 20000)
    assert gg.graph_sha256(a) == gg.graph_sha256(b)
    key = a.eu.astype(np.int64) * a.n_v + a.ev
    assert np.unique(key).shape[0] == a.m
    assert a.eu.dtype == np.int32 and a.ev.dtype == np.int32
    assert a.eu.min() >= 0 and a.eu.max() < a.n_u and a.ev.max() < a.n_v


def test_chung_lu_is_skewed_and_seeded():
    g = gg.chung_lu(20000, 4000, 200000, 2.5, 2.1, seed=3, cap_v=2000)
    h = gg.chung_lu(20000, 4000, 200000, 2.5, 2.1, seed=3, cap_v=2000)
    k = gg.chung_lu(20000, 4000, 200000, 2.5, 2.1, seed=4, cap_v=2000)
    assert gg.graph_sha256(g) == gg.graph_sha256(h) != gg.graph_sha256(k)
    dv = np.bincount(g.ev, minlength=g.n_v)
    du = np.bincount(g.eu, minlength=g.n_u)
    assert 0.9 * 200000 < g.m <= 200000
    assert dv.max() > 20 * dv.mean()          # hubs on V
    assert dv.max() <= 2000 * 1.5             # cap respected up to sampling noise
    assert du.max() > 10 * du.mean()


def test_batch_and_serving_params():
    ps = gg.batch_params()
    assert len(ps) == 64
    assert all(1e4 * 0.99 <= p["m_t"] <= 2e6 * 1.01 for p in ps)
    assert all(1.0 <= p["n_u"] / p["n_v"] <= 8.2 for p in ps)
    assert ps == gg.batch_params()
    tr = gg.serving_trace(duration=10.0)
    assert 100 < len(tr) < 320
    assert all(a["arrival"] < b["arrival"] for a, b in zip(tr, tr[1:]))
    assert {j["side"] for j in tr} == {0, 1}


def test_permute_and_transpose():
    g = gg.tiny_random(9, 7, 0.5, 1)
    gp, pu, pv = gg.permute_ids(g, 2)
    assert gp.m == g.m
    assert set(zip(gp.eu.tolist(), gp.ev.tolist())) == \
        set(zip(pu[g.eu].tolist(), pv[g.ev].tolist()))
    gt = gg.transpose(g)
    assert (gt.n_u, gt.n_v) == (g.n_v, g.n_u)
    assert set(zip(gt.eu.tolist(), gt.ev.tolist())) == set(zip(g.ev.tolist(), g.eu.tolist()))
