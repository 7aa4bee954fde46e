"""GPU parity of the batched executor: many star queries of uneven sizes run as
one instance-prefixed arena, eagerly and as a replayed HIP graph, each
instance bit-exact against the CPU oracle's statement of that query; plus the
autotuner (knobs change launch shapes, never results)."""
import numpy as np
import pytest

import oracle
import tqp_datagen as dg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def to_dev(tbl):
    return {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in tbl.items()}


def dev_instances(insts):
    return [{"fact": to_dev(i["fact"]), "dim": to_dev(i["dim"])} for i in insts]


def check_against_oracle(insts, got):
    assert len(got) == len(insts)
    for k, (inst, g) in enumerate(zip(insts, got)):
        want = oracle.q1(inst["fact"], inst["dim"], inst["day_cut"])
        assert not want["overflow"]
        for name in ("key", "sum_qty", "count"):
            assert np.array_equal(np.asarray(g[name], dtype=np.int64),
                                  np.asarray(want[name], dtype=np.int64)), (k, name)


def test_batch_uneven_sizes_match_oracle():
    from paper_2209_04579_amd.batch import BatchStarQuery
    insts = dg.config5(0, instances=12, fact_lo=100, fact_hi=300_000)
    b = BatchStarQuery(dev_instances(insts), 1278)
    b.run()
    check_against_oracle(insts, b.results())


def test_batch_graph_replays_match_oracle_and_sequential():
    from paper_2209_04579_amd.batch import BatchStarQuery, SequentialStarQueries
    insts = dg.config5(1, instances=9, fact_lo=1000, fact_hi=200_000)
    dev = dev_instances(insts)
    b = BatchStarQuery(dev, 1278)
    b.capture()
    seq = SequentialStarQueries(dev, 1278)
    seq.run()
    want = seq.results()
    check_against_oracle(insts, want)
    for _ in range(3):
        b.run()
        got = b.results()
        check_against_oracle(insts, got)
        # eager work between replays
        seq.run()
        torch.cuda.synchronize()


def test_batch_degenerate_instances():
    from paper_2209_04579_amd.batch import BatchStarQuery
    insts = []
    for seed, nf, nd in [(0, 0, 5), (1, 1, 1), (2, 3000, 1), (3, 5, 3), (4, 70_000, 4000)]:
        c = dg.config1(seed, n_fact=nf, n_dim=nd)
        insts.append(c)
    b = BatchStarQuery(dev_instances(insts), 1278)
    b.run()
    check_against_oracle(insts, b.results())


def test_tuning_changes_nothing_but_time():
    from paper_2209_04579_amd import autotune, tune_knobs, tune_set
    from paper_2209_04579_amd.pipeline import StarQuery
    cfg = dg.config2(0, n_fact=400_000, n_dim=20_000)
    fact, dim = to_dev(cfg["fact"]), to_dev(cfg["dim"])
    want = oracle.q2(cfg["fact"], cfg["dim"], cfg["day_cut"])
    defaults = {k: v[0] for k, v in tune_knobs().items()}
    try:
        best, ms, timings = autotune.tune(lambda t: StarQuery(fact, dim, cfg["day_cut"], "q2", t),
                                          reps=1, rounds=1)
        assert ms > 0 and len(timings) >= len(defaults)
        knobs = tune_knobs()
        for k, v in best.items():
            if k in knobs:
                assert knobs[k][1] <= v <= knobs[k][2]
        # extreme settings: every knob at its low end, then its high end
        for end in (1, 2):
            t = {k: v[end] for k, v in knobs.items()}
            t["gb.dense_max"] = 0 if end == 1 else 1024
            q = StarQuery(fact, dim, cfg["day_cut"], "q2", t)
            q.run()
            got = q.result()
            for name in ("a_key", "a_qty", "a_price", "a_count", "b_key", "b_qty", "b_count"):
                assert np.array_equal(got[name], want[name]), (end, name)
    finally:
        for k, v in defaults.items():
            tune_set(k, v)


@pytest.mark.timeout(900)
def test_batch_full_size_matches_oracle():
    """256 instances at full size (633M fact rows, drawn on the GPU), captured
    in a graph, every instance against the oracle on host copies."""
    from paper_2209_04579_amd.batch import BatchStarQuery
    from tqp_datagen import device as dgd
    dev = dgd.config5(0, device="cuda")
    b = BatchStarQuery([{"fact": i["fact"], "dim": i["dim"]} for i in dev], 1278)
    b.capture()
    b.run()
    got = b.results()
    del b
    torch.cuda.empty_cache()
    insts = [{"fact": {k: v.cpu().numpy() for k, v in i["fact"].items()},
              "dim": {k: v.cpu().numpy() for k, v in i["dim"].items()},
              "day_cut": 1278} for i in dev]
    check_against_oracle(insts, got)


@pytest.mark.parametrize("kdt", [np.int32, np.int64])
@pytest.mark.parametrize("n", [0, 1, 5000, 1_000_003])
def test_lower_bound_matches_searchsorted(kdt, n):
    import paper_2209_04579_amd as tqp
    keys = np.sort(dg.uniform_int(n + 1, 1, n, -1000, 1000, kdt))
    q = np.concatenate([dg.uniform_int(n + 2, 2, 997, -1100, 1100, np.int64),
                        np.array([np.iinfo(np.int64).min, np.iinfo(np.int64).max, 0])])
    out = torch.empty(len(q), dtype=torch.int64, device="cuda")
    d_n = torch.tensor([n // 2], dtype=torch.int64, device="cuda")
    tqp.lower_bound_into(torch.from_numpy(keys).cuda(), torch.from_numpy(q).cuda(), out, d_n=d_n)
    assert np.array_equal(out.cpu().numpy(), np.searchsorted(keys[:n // 2], q, side="left"))
    tqp.lower_bound_into(torch.from_numpy(keys).cuda(), torch.from_numpy(q).cuda(), out)
    assert np.array_equal(out.cpu().numpy(), np.searchsorted(keys, q, side="left"))
