"""GPU parity for PREDICT inside a query (tqp_mlp_predict, Section 3.3's
prediction queries): the class of every row equals the oracle's, which takes
the same fp32 fused multiply-adds in the same order, over models of every
supported shape, every feature dtype, with and without row ids; then the
whole prediction query (filter, score, GROUP BY rating with a CASE count)
against the oracle up to 20M rows."""
import numpy as np
import pytest

import oracle
import tqp_datagen as dg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tqp():
    import paper_2209_04579_amd as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def predict(tqp, feats, model, H, C, rows=None):
    n = len(rows) if rows is not None else len(feats[0])
    out = torch.full((max(n, 1),), -1, dtype=torch.int8, device="cuda")
    tqp.mlp_predict_into([dev(f) for f in feats], dev(model), H, C, out, n=n,
                         rows=None if rows is None else dev(rows))
    torch.cuda.synchronize()
    return out[:n].cpu().numpy()


@pytest.mark.parametrize("F,H,C", [(1, 1, 1), (3, 5, 2), (8, 16, 2), (16, 64, 8), (7, 33, 3)])
@pytest.mark.parametrize("n", [0, 1, 257, 100_003])
def test_predict_matches_oracle(tqp, F, H, C, n):
    seed = F * 100 + H + C
    model = dg.mlp_model(seed, F, H, C)
    dts = [np.int8, np.int32, np.int64]
    feats = [dg.uniform_int(seed, 20 + k, n, -30, 31, dts[k % 3]) for k in range(F)]
    assert np.array_equal(predict(tqp, feats, model, H, C), oracle.mlp_predict(feats, model, H, C))


def test_predict_through_row_ids_and_zero_rows(tqp):
    cfg = dg.config_predict(4, 50_000)
    F, H = cfg["nfeat"], cfg["hidden"]
    feats = [cfg["reviews"][f"f{k}"] for k in range(F)]
    rows = dg.uniform_int(4, 99, 30_001, 0, 50_000, np.int32)
    got = predict(tqp, feats, cfg["model"], H, 2, rows)
    assert np.array_equal(got, oracle.mlp_predict(feats, cfg["model"], H, 2, rows))
    # a row id outside the columns reads zero features
    bad = np.array([-1, 50_000, 7], np.int32)
    zero = [np.zeros(1, f.dtype) for f in feats]
    z = oracle.mlp_predict(zero, cfg["model"], H, 2)[0]
    assert predict(tqp, feats, cfg["model"], H, 2, bad).tolist() == \
        [z, z, oracle.mlp_predict(feats, cfg["model"], H, 2, bad[2:])[0]]


def test_predict_exact_integer_model(tqp):
    F, H, C, n = 6, 9, 4, 20_000
    model = dg.uniform_int(8, 30, H * F + H + C * H + C, -4, 5, np.int64).astype(np.float32)
    feats = [dg.uniform_int(8, 40 + k, n, -6, 7, np.int32) for k in range(F)]
    assert np.array_equal(predict(tqp, feats, model, H, C), oracle.mlp_predict(feats, model, H, C))


def run_query(cfg, reviews=None):
    from paper_2209_04579_amd.pipeline import PredictQuery
    reviews = reviews or {k: dev(v) for k, v in cfg["reviews"].items()}
    q = PredictQuery(reviews, cfg["model"], cfg["nfeat"], cfg["hidden"], cfg["classes"],
                     cfg["year_min"], cfg["nratings"])
    q.run()
    return q, q.result()


@pytest.mark.parametrize("seed,n", [(0, 2_000_000), (1, 1), (2, 4_097)])
def test_predict_query_matches_oracle(tqp, seed, n):
    cfg = dg.config_predict(seed, n)
    q, got = run_query(cfg)
    want = oracle.q_predict(cfg)
    assert np.array_equal(got["count"], want["count"])
    assert np.array_equal(got["positive"], want["positive"])
    q.run()
    again = q.result()
    assert np.array_equal(again["positive"], got["positive"])


def test_predict_query_full_size(tqp):
    from tqp_datagen import device as dgd
    d = dgd.config_predict(0, device="cuda")
    _, got = run_query(d, d["reviews"])
    host = dict(d, reviews={k: v.cpu().numpy() for k, v in d["reviews"].items()})
    want = oracle.q_predict(host)
    assert np.array_equal(got["count"], want["count"]) and got["count"].sum() > 0
    assert np.array_equal(got["positive"], want["positive"])
