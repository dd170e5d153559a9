"""Host-side logic of the generator, router and autotuner (no GPU).

The class kernels' numerics are checked against the oracle on the GPU; these
tests pin what can be checked without one: the VRR graph's structure and
schedules (Sec. III-A), the generator's T^(l) against the oracle's
independent closed form, the router's table/model merge, the tuner's
selection, and the lane-index logic of the segmented wave reduction used by
the J/K digestion (run on a 64-lane emulation)."""
import json

import numpy as np
import pytest

import oracle
from paper_2605_10312_amd.gen import cart, router, vrr
from paper_2605_10312_amd.gen import sph as gsph


@pytest.mark.parametrize("ls", [(0, 0, 0, 0), (1, 0, 1, 0), (2, 1, 1, 0), (2, 2, 2, 2)])
def test_vrr_graph_targets_and_orders(ls):
    g = vrr.VRRGraph(*ls)
    la, lb, lc, ld = ls
    # targets [e0|f0] with la <= |e| <= la+lb, lc <= |f| <= lc+ld
    n_e = sum(cart.ncart(e) for e in range(la, la + lb + 1))
    n_f = sum(cart.ncart(f) for f in range(lc, lc + ld + 1))
    assert g.n_hrr() == n_e * n_f
    # base nodes: one per order m = 0..L
    base = [nd for nd in g.nodes if nd.kind == "base"]
    assert sorted(nd.key[2] for nd in base) == list(range(len(base)))
    assert len(base) <= g.L + 1
    for name, fn in vrr.SCHEDULERS.items():
        order = fn(g)
        assert sorted(order) == list(range(len(g.nodes))), name     # every node once
        pos = {v: i for i, v in enumerate(order)}
        for v, nd in enumerate(g.nodes):                              # parents before children
            for p in nd.parents:
                if p is not None:
                    assert pos[p] < pos[v], name
        assert 0 <= vrr.peak_live(g, order) <= len(g.nodes)
    sched, pl, order = vrr.best_order(g)
    assert pl == min(vrr.peak_live(g, fn(g)) for fn in vrr.SCHEDULERS.values())


def test_vrr_node_keys_follow_the_recurrence():
    """Every non-base node (e, f, m) lowers exactly one index of e (bra step) or
    f (ket step) by one and draws on orders m and m + 1 only."""
    g = vrr.VRRGraph(2, 1, 2, 0)
    for nd in g.nodes:
        if nd.kind == "base":
            assert sum(nd.key[0]) == 0 and sum(nd.key[1]) == 0
            continue
        e, f, m = nd.key
        p1 = g.nodes[nd.parents[0]].key
        side = 0 if nd.kind == "bra" else 1
        lowered = (e, f)[side]
        assert sum(lowered) - sum(p1[side]) == 1
        assert p1[2] in (m, m + 1)
        for p in nd.parents:
            if p is not None:
                assert g.nodes[p].key[2] in (m, m + 1)


@pytest.mark.parametrize("l", [0, 1, 2, 3, 4])
def test_generator_tmatrix_matches_oracle(l):
    """The generator's T^(l) (sympy, exact) and the oracle's (C closed form)
    are written independently; they must agree entry by entry."""
    assert np.allclose(gsph.tmatrix_dense(l), oracle.sph_matrix(l), rtol=0, atol=1e-14)


def test_canonical_class_counts():
    assert [len(cart.canonical_classes(l)) for l in (2, 3, 4)] == [21, 55, 120]


def test_router_table_overrides_model(tmp_path):
    ls = (2, 2, 2, 1)
    model = router.route(ls, {})
    assert model["source"] == "model" and model["tier"] == 1 and model["cap"] in router.CAPS
    # a measured entry wins; what it leaves out comes from the model
    r = router.route(ls, {"2221": {"tier": 1, "reduce": "none", "variant": "x", "ms": 1.0}})
    assert r["source"] == "table" and r["reduce"] == "none" and r["cap"] == model["cap"]
    assert "variant" not in r and "ms" not in r
    r = router.route((1, 0, 0, 0), {"1000": {"tier": 0, "waves": 2}})
    assert r["tier"] == 0 and r["waves"] == 2
    assert router.route((1, 0, 0, 0), {})["tier"] == 0


def test_tuner_select(tmp_path, monkeypatch):
    from paper_2605_10312_amd import tune
    monkeypatch.setattr(tune, "VARIANTS", {"a": {"reduce": "none"}, "b": {"reduce": "segmented", "waves": 2,
                                                                        "digest": "interleaved"}})
    res = {"a": {"ms_per_build": 3.0, "classes": {"1000": {"tier": 0, "ms": 1.0}, "2222": {"tier": 1, "ms": 2.0}}},
           "b": {"ms_per_build": 2.5, "classes": {"1000": {"tier": 0, "ms": 1.5}, "2222": {"tier": 1, "ms": 1.0}}}}
    path = tmp_path / "r.json"
    path.write_text(json.dumps(res))
    table = tmp_path / "t.json"
    monkeypatch.setattr(tune, "VARIANTS_DIR", str(tmp_path))
    clean = {"jk_1000": {"scratch": 0}, "p1_2222": {"scratch": 0}, "jk_2222": {"scratch": 0}}
    for v in ("a", "b"):
        (tmp_path / f"libhgp_{v}.resources.json").write_text(json.dumps(clean))
    tune.select(str(path), table=str(table))
    got = json.loads(table.read_text())["classes"]
    assert got["1000"]["variant"] == "a" and got["1000"]["reduce"] == "none"
    # a staged class keeps only the options its emitter takes
    assert got["2222"]["variant"] == "b" and got["2222"]["waves"] == 2 and "digest" not in got["2222"]
    # a variant that compiled the class with private scratch is never chosen, however fast
    spill = dict(clean, p1_2222={"scratch": 16})
    (tmp_path / "libhgp_b.resources.json").write_text(json.dumps(spill))
    tune.select(str(path), table=str(table))
    got = json.loads(table.read_text())["classes"]
    assert got["2222"]["variant"] == "a"


def test_router_fallback_ladder():
    from paper_2605_10312_amd.gen import router
    assert router.fallback({"tier": 0}, ["jk_2120"]) == {"tier": 1}
    assert router.fallback({"tier": 1, "cap": 96}, ["p1_2222"]) == {"tier": 1, "cap": 64}
    assert router.fallback({"tier": 1, "cap": 16}, ["p1_2222"]) == {"tier": 2}
    # a J/K kernel that spills with the one-pass digestion goes back to the six-pass form first
    assert router.fallback({"tier": 1, "cap": 96}, ["jk_4410", "p1_4410"]) == \
        {"tier": 1, "cap": 96, "jk_digest": "slots"}
    assert router.fallback({"tier": 1, "cap": 96, "jk_digest": "slots"}, ["jk_4410", "p1_4410"]) == {"tier": 2}
    assert router.fallback({"tier": 1, "cap": 96, "jk_digest": "slots"}, ["p1_4410"]) == \
        {"tier": 1, "cap": 64, "jk_digest": "slots"}
    assert router.fallback({"tier": 2}, ["t3_jk_kernel"]) is None
    assert router.fallback({"tier": 1, "form": "row", "budget": 240}, ["p1_3333"]) == \
        {"tier": 1, "form": "row", "budget": 220}
    assert router.fallback({"tier": 1, "form": "row", "budget": 220}, ["p1_3333p3"]) == \
        {"tier": 1, "form": "row", "budget": 200}
    assert router.fallback({"tier": 1, "form": "row", "budget": 160}, ["p1_3333"]) == {"tier": 2}
    assert router.fallback({"tier": 1, "form": "row", "budget": 240}, ["jk_4444"]) == \
        {"tier": 1, "form": "row", "budget": 240, "jk_digest": "slots"}
    assert router.fallback({"tier": 1, "form": "row", "budget": 240, "jk_digest": "slots"}, ["jk_4444"]) == \
        {"tier": 2}
    assert router.route((3, 3, 3, 3), {})["form"] == "row" and router.route((2, 2, 2, 1), {})["form"] == "chunk"
    assert router.route((4, 3, 2, 1), {})["form"] == "row"
    assert router.route((4, 4, 2, 1), {})["tier"] == 2             # a (gg| bra stays on the op tables
    assert router.route((4, 4, 4, 3), {})["tier"] == 2             # a (gg| ket: rows of 145 do not fit


def test_resource_remarks_parse():
    from paper_2605_10312_amd import build
    err = "\n".join([
        "x.hip:3:1: remark: Function Name: _ZN3hgp12_GLOBAL__N_17jk_2120ENS_6JKArgsE [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:3:1: remark:     VGPRs: 256 [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:3:1: remark:     AGPRs: 121 [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:3:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:3:1: remark:     Dynamic Stack: False [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:3:1: remark:     Occupancy [waves/SIMD]: 1 [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:9:1: remark: Function Name: _ZN3hgp12_GLOBAL__N_114t3w_eri_kernelILb0EEEvNS_7EriArgsE "
        "[-Rpass-analysis=kernel-resource-usage]",
        "x.hip:9:1: remark:     ScratchSize [bytes/lane]: 24 [-Rpass-analysis=kernel-resource-usage]",
    ])
    res = build.parse_resource_remarks(err)
    assert res["jk_2120"]["vgpr"] == 256 and res["jk_2120"]["agpr"] == 121 and res["jk_2120"]["occupancy"] == 1
    assert res["jk_2120"]["dynamic_stack"] is False
    assert build.check_resources(res) == ["t3w_eri_kernel<false>"]
    assert build.class_scratch(res, "2120") == 0
    # Phase-1 parts of a row-form class count for their class
    assert build._spilled_classes({"p1_3333p2": {"scratch": 8}, "jk_3333": {"scratch": 0},
                                   "jk_2120": {"scratch": 4}}) == {"3333": ["p1_3333p2"], "2120": ["jk_2120"]}
    assert build.class_scratch({"p1_3333p1": {"scratch": 12}}, "3333") == 12


def test_generate_applies_defaults_and_overrides(tmp_path):
    from paper_2605_10312_amd import build
    files, metas = build.generate(1, gen_dir=str(tmp_path), table={}, defaults={"reduce": "none"},
                                  overrides={"1010": {"reduce": "segmented"}})
    src = {m.tag: open(tmp_path / f"class_{m.tag}.hip").read() for m in metas}
    assert len(metas) == len(cart.canonical_classes(1))
    assert "hgp_seg_sum" in src["1010"] and "hgp_seg_sum" not in src["1000"]
    assert all(m.tier == 0 for m in metas)
    assert (tmp_path / "class_table.hip").exists()


# --- the segmented reduction's lane logic, emulated on 64 lanes -------------

def _shfl_up(v, o):
    return np.array([v[i - o] if i >= o else v[i] for i in range(64)])


def _seg_start(key, active):
    lane = np.arange(64)
    prev = _shfl_up(key, 1)
    s = np.where((lane == 0) | (prev != key), lane, 0)
    o = 1
    while o < 64:
        t = _shfl_up(s, o)
        s = np.where(lane >= o, np.maximum(s, t), s)
        o <<= 1
    return s


def _seg_tail(key, active):
    nxt = np.array([key[i + 1] if i < 63 else key[i] for i in range(64)])
    live_next = np.array([active[i + 1] if i < 63 else False for i in range(64)])
    return (np.arange(64) == 63) | ~live_next | (nxt != key)


def _seg_sum(v, start):
    lane = np.arange(64)
    o = 1
    while o < 64:
        t = _shfl_up(v, o)
        v = np.where(lane - o >= start, v + t, v)
        o <<= 1
    return v


@pytest.mark.parametrize("seed", range(20))
def test_segmented_reduction_lane_logic(seed):
    """Runs of equal keys (as in the sorted quartet lists), an active prefix
    of the wave (a list's last wave), random values: the run-tail lanes must
    hold exactly the run sums, so that their atomics add every active lane's
    value once."""
    rng = np.random.default_rng(seed)
    nact = 64 if seed % 3 else int(rng.integers(1, 64))
    runs = rng.integers(1, 20, 64)
    # runs of equal keys; a key may come back in a later run (two atomics then)
    key = np.repeat(rng.integers(0, 5, 64), runs)[:64] * 7 + 3
    active = np.arange(64) < nact
    v = rng.normal(size=64)
    start = _seg_start(key, active)
    tail = _seg_tail(key, active) & active
    tot = _seg_sum(v, start)
    got = {}
    for i in np.nonzero(tail)[0]:
        got[key[i]] = got.get(key[i], 0.0) + tot[i]
    want = {}
    for i in range(nact):
        want[key[i]] = want.get(key[i], 0.0) + v[i]
    assert set(got) == set(want)
    for k in want:
        assert abs(got[k] - want[k]) <= 1e-12 * max(1.0, abs(want[k]))
