"""GPU parity of the learned CDF partitioner: the partition sort gives the same
bytes as the radix sort and the oracle's stable sort whatever the model, the
model is monotone (buckets are key ranges), a degenerate model forces the
radix fallback and still sorts exactly, and a join over partition-sorted
sides gives the oracle's ranges."""
import numpy as np
import pytest

import oracle
import tqp_datagen as dg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tqp():
    import paper_2209_04579_amd as m
    assert torch.cuda.is_available()
    m.lib()
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def mix():
    c = dg.config4(0, n_left=2_000_000, n_right=500_000)
    return c["left"], c["right"]


def test_model_is_monotone_and_trains(tqp, mix):
    left, right = mix
    model = tqp.lcdf_train([dev(left), dev(right)], sample_stride=100, nleaf=4096, steps=100)
    info = tqp.lcdf_model_info(model)
    assert info["nleaf"] == 4096 and info["steps"] == 100
    assert info["loss_best"] < info["loss_first"]        # training improved the root
    assert info["loss_last"] <= info["loss_first"]       # and did not diverge
    sk = np.sort(np.concatenate([left, right]))
    b = host(tqp.lcdf_buckets(model, dev(sk), 16))
    assert np.all(np.diff(b) >= 0), "bucket numbers must not decrease along sorted keys"
    assert b.min() >= 0 and b.max() < 65536
    # extremes of the key domain stay in range
    ext = np.array([np.iinfo(np.int64).min, -1, 0, np.iinfo(np.int64).max], np.int64)
    eb = host(tqp.lcdf_buckets(model, dev(ext), 16))
    assert np.all(np.diff(eb) >= 0) and eb.min() >= 0 and eb.max() < 65536


@pytest.mark.parametrize("nleaf", [1, 1688, 1689, 3 * 1688 + 5])
def test_bucket_numbers_every_leaf_group(tqp, mix, nleaf):
    """Bucket numbers are evaluated with the leaves in LDS, one group of 1688
    leaves per pass over the keys: every key gets its number in exactly one
    pass (a pre-filled output is overwritten everywhere), numbers do not
    decrease along sorted keys, and the partition sort is the stable sort."""
    left, right = mix
    model = tqp.lcdf_train([dev(left), dev(right)], sample_stride=50, nleaf=nleaf, steps=20)
    sk = np.sort(np.concatenate([left, right]))
    out = torch.full((sk.size,), -1, dtype=torch.int32, device="cuda")
    b = host(tqp.lcdf_buckets(model, dev(sk), 16, out=out))
    assert b.min() >= 0 and b.max() < 65536
    assert np.all(np.diff(b) >= 0)
    got, rows, _ = tqp.partition_sort(dev(right), tqp.PART_LEARNED, model, bucket_bits=14)
    ok, perm = oracle.sort(right)
    assert np.array_equal(host(got), ok) and np.array_equal(host(rows), perm)


@pytest.mark.parametrize("bits", [8, 12, 16, 20, 24])
def test_learned_partition_sort_matches_sort_and_oracle(tqp, mix, bits):
    left, right = mix
    model = tqp.lcdf_train([dev(left), dev(right)], steps=50)
    for keys in (left, right):
        sk, rows, st = tqp.partition_sort(dev(keys), tqp.PART_LEARNED, model, bucket_bits=bits)
        ok, perm = oracle.sort(keys)
        assert np.array_equal(host(sk), ok)
        assert np.array_equal(host(rows), perm)
        assert st["max_bucket"] >= 1


@pytest.mark.parametrize("bits", [4, 12, 16, 24])
def test_msd_radix_partition_sort_matches(tqp, mix, bits):
    left, _ = mix
    sk, rows, st = tqp.partition_sort(dev(left), tqp.PART_RADIX, None, bucket_bits=bits)
    ok, perm = oracle.sort(left)
    assert np.array_equal(host(sk), ok) and np.array_equal(host(rows), perm)
    assert st["fallback_buckets"] >= 1          # clusters and lognormal mass overflow


def test_degenerate_model_forces_fallback(tqp):
    const = np.full(10_000, 77, np.int64)
    model = tqp.lcdf_train([dev(const)], sample_stride=10, nleaf=16, steps=5)
    keys = dg.uniform_int(3, 1, 300_000, -10 ** 6, 10 ** 6, np.int64)
    sk, rows, st = tqp.partition_sort(dev(keys), tqp.PART_LEARNED, model, bucket_bits=12)
    ok, perm = oracle.sort(keys)
    assert np.array_equal(host(sk), ok) and np.array_equal(host(rows), perm)
    assert st["fallback_buckets"] >= 1 and st["fallback_keys"] >= 300_000 // 2


@pytest.mark.parametrize("n", [0, 1, 5, 4097, 100_003])
def test_partition_sort_small_and_int32(tqp, n):
    keys = dg.uniform_int(n + 1, 1, n, -50, 50, np.int32)
    src = keys if n >= 2 else np.array([1, 2], np.int32)
    model = tqp.lcdf_train([dev(src)], sample_stride=1, nleaf=64, steps=10)
    for mode, mdl in ((tqp.PART_LEARNED, model), (tqp.PART_RADIX, None)):
        sk, rows, _ = tqp.partition_sort(dev(keys), mode, mdl, bucket_bits=6)
        ok, perm = oracle.sort(keys)
        assert np.array_equal(host(sk), ok) and np.array_equal(host(rows), perm)


def test_heavy_duplicates_single_valued_buckets(tqp):
    # one key holds 60% of the rows: its bucket is single-valued and kept as is
    keys = dg.uniform_int(5, 1, 400_000, 0, 10 ** 9, np.int64)
    keys[dg.uniform_float(5, 2, 400_000) < 0.6] = 123_456_789
    model = tqp.lcdf_train([dev(keys)], steps=20)
    sk, rows, st = tqp.partition_sort(dev(keys), tqp.PART_LEARNED, model, bucket_bits=12)
    ok, perm = oracle.sort(keys)
    assert np.array_equal(host(sk), ok) and np.array_equal(host(rows), perm)
    assert st["single_valued_big"] >= 1


def test_join_ranges_over_partition_sorted_sides(tqp, mix):
    left, right = mix
    model = tqp.lcdf_train([dev(left), dev(right)], steps=50)
    sl, _, _ = tqp.partition_sort(dev(left), tqp.PART_LEARNED, model, bucket_bits=12)
    sr, _, _ = tqp.partition_sort(dev(right), tqp.PART_LEARNED, model, bucket_bits=12)
    got = tqp.join_ranges(sl, sr)
    want = oracle.join_ranges(left, right)
    for k in ("key", "lstart", "lcnt", "rstart", "rcnt"):
        assert np.array_equal(host(got[k]), want[k]), k
    assert got["total"] == want["total"]


def assert_stable_sort(keys, sk, rows):
    """The four properties that together define the stable ascending sort:
    sk is non-decreasing, sk = keys[rows], rows is a permutation, and rows
    increase along runs of equal keys."""
    n = keys.numel()
    assert sk.numel() == n and rows.numel() == n
    if n == 0:
        return
    assert bool(torch.all(sk[1:] >= sk[:-1]))
    r = rows.long()
    assert bool(torch.all((r >= 0) & (r < n)))
    assert torch.equal(keys[r], sk)
    assert bool(torch.all(torch.bincount(r, minlength=n) == 1))
    eq = sk[1:] == sk[:-1]
    assert bool(torch.all(r[1:][eq] > r[:-1][eq]))


@pytest.mark.timeout(900)
def test_full_size_learned_join_matches_oracle(tqp):
    """200M x 50M int64 keys at full size, in the benchmark's setting: the
    learned partition sort of each side is the stable sort (property check on
    the device), and the join ranges over the sorted sides equal the oracle's
    on host copies."""
    from tqp_datagen import device as dgd
    c = dgd.config4(0, device="cuda")
    left, right = c["left"], c["right"]
    # the benchmark's setting: 1688 leaves, 50 steps, 2^16 buckets
    model = tqp.lcdf_train([left, right], sample_stride=100, nleaf=1688, steps=50)
    sides = []
    for keys in (left, right):
        sk, rows, st = tqp.partition_sort(keys, tqp.PART_LEARNED, model, bucket_bits=16)
        assert st["fallback_keys"] < 0.01 * keys.numel()
        assert_stable_sort(keys, sk, rows)
        del rows
        sides.append(sk)
    got = tqp.join_ranges(sides[0], sides[1])
    want = oracle.join_ranges(host(left), host(right))
    for k in ("key", "lstart", "lcnt", "rstart", "rcnt"):
        assert np.array_equal(host(got[k]), want[k]), k
    assert got["total"] == want["total"]


def test_heavy_keys_get_buckets_of_their_own(tqp, mix):
    """Zipf heavy hitters fill whole buckets; the model's jumps at heavy keys
    keep them out of multi-valued buckets, so little goes to the fallback,
    unlike the MSD radix partition of the same keys."""
    left, right = mix
    n = left.size
    bits = max(1, (n // 1024).bit_length())
    model = tqp.lcdf_train([dev(left), dev(right)], sample_stride=100, nleaf=4096, steps=200)
    sk, rows, st = tqp.partition_sort(dev(left), tqp.PART_LEARNED, model, bucket_bits=bits)
    ok, perm = oracle.sort(left)
    assert np.array_equal(host(sk), ok) and np.array_equal(host(rows), perm)
    assert st["single_valued_big"] >= 1
    sk2, rows2, st2 = tqp.partition_sort(dev(left), tqp.PART_RADIX, None, bucket_bits=bits)
    assert np.array_equal(host(sk2), ok) and np.array_equal(host(rows2), perm)
    assert st["fallback_keys"] < 0.05 * n
    assert st["fallback_keys"] < st2["fallback_keys"]


def test_overflow_cap_sorts_whole_input(tqp, mix):
    """With the overflow cap at 1 and several overflowing buckets, the whole
    input goes through the plain radix sort; the result is the same."""
    left, _ = mix
    old = tqp.tune_knobs()["part.ovf_cap"][0]
    try:
        tqp.tune_set("part.ovf_cap", 1)
        sk, rows, st = tqp.partition_sort(dev(left), tqp.PART_RADIX, None, bucket_bits=8)
        assert st["fallback_buckets"] >= 2
        ok, perm = oracle.sort(left)
        assert np.array_equal(host(sk), ok) and np.array_equal(host(rows), perm)
    finally:
        tqp.tune_set("part.ovf_cap", old)
