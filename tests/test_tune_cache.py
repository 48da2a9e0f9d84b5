"""Host side of the batch autotune cache (rz_tune_cache_*, rz_order_class_host
in include/rz.h): the cache file's round trip, its handling of malformed and
concurrent input, and the point-order classifier of its key.  No GPU."""
import os
import threading

import numpy as np
import pytest

from paper_1908_02681_amd import gen


@pytest.fixture(scope="module")
def rz():
    from paper_1908_02681_amd import rz as binding
    binding.load()
    return binding


KEY = "gfx950 n27 px26 v64 hq4 ordered"
DEPTH = {"block": 64, "ppt": 16, "early_out": 1, "xcd_remap": 0, "bin": 2}
ACCUM = {"block": 128, "ppt": 8, "early_out": 1, "xcd_remap": 1, "bin": 2}


def test_missing_file_is_a_miss(rz, tmp_path):
    assert rz.tune_cache_lookup(str(tmp_path / "none.txt"), KEY) is None


def test_round_trip_and_replace(rz, tmp_path):
    path = str(tmp_path / "c.txt")
    rz.tune_cache_store(path, KEY, 4, DEPTH, ACCUM, 27.8125)
    e = rz.tune_cache_lookup(path, KEY)
    assert e == {"views_per_group": 4, "depth": DEPTH, "accum": ACCUM, "ms": 27.8125}
    other = KEY.replace("ordered", "shuffled")
    assert rz.tune_cache_lookup(path, other) is None
    rz.tune_cache_store(path, other, 8, ACCUM, DEPTH, 1.5)
    d2 = dict(DEPTH, block=256, ppt=4)
    rz.tune_cache_store(path, KEY, 2, d2, ACCUM, 20.0)   # replaces the first line
    assert rz.tune_cache_lookup(path, KEY) == {"views_per_group": 2, "depth": d2,
                                               "accum": ACCUM, "ms": 20.0}
    assert rz.tune_cache_lookup(path, other)["views_per_group"] == 8
    lines = [l for l in open(path).read().splitlines() if not l.startswith("#")]
    assert len(lines) == 2 and sum(l.startswith(KEY + " ") for l in lines) == 1
    assert not [f for f in os.listdir(tmp_path) if ".tmp." in f]


def test_malformed_lines_are_ignored_and_dropped(rz, tmp_path):
    path = str(tmp_path / "c.txt")
    good = (f"{KEY} k=4 block=64 ppt=16 early_out=1 xcd=0 bin=2 hq_block=128 hq_ppt=8 "
            "hq_early_out=1 hq_xcd=1 hq_bin=2 ms=3.5")
    bad = [
        "garbage",
        f"{KEY} k=4",                                              # fields missing
        good.replace("k=4", "k=9"),                                # K out of range
        good.replace("block=64", "block=96"),                      # not a block size
        good.replace("ms=3.5", "ms=nan"),
        good.replace("ppt=16", "ppt=16x"),
        good + " extra=1",                                         # unknown field
        good.replace("bin=2 hq", "bin2 hq"),                       # no '='
    ]
    with open(path, "w") as f:
        f.write("# comment\n\n" + "\n".join(bad) + "\n")
    assert rz.tune_cache_lookup(path, KEY) is None
    with open(path, "a") as f:
        f.write(good + "\n")
    e = rz.tune_cache_lookup(path, KEY)
    assert e["views_per_group"] == 4 and e["accum"]["xcd_remap"] == 1 and e["ms"] == 3.5
    rz.tune_cache_store(path, "gfx950 n20 px20 v8 hq0 shuffled", 1, DEPTH, DEPTH, 0.25)
    body = [l for l in open(path).read().splitlines() if l and not l.startswith("#")]
    assert len(body) == 2 and good in body   # the bad lines are gone, the good one kept


@pytest.mark.parametrize("key", ["", "a b c d e", "a b c d e f g", " a b c d e f",
                                 "a b c d e f ", "a  b c d e f", "a b c d e f\n", "a\tb c d e f"])
def test_bad_keys_are_refused(rz, tmp_path, key):
    path = str(tmp_path / "c.txt")
    with pytest.raises(rz.RzError) as ei:
        rz.tune_cache_store(path, key, 4, DEPTH, ACCUM, 1.0)
    assert ei.value.code == rz.RZ_EINVAL
    with pytest.raises(rz.RzError):
        rz.tune_cache_lookup(path, key)
    assert not os.path.exists(path)


@pytest.mark.parametrize("k,depth,ms", [(0, DEPTH, 1.0), (9, DEPTH, 1.0),
                                        (4, dict(DEPTH, block=32), 1.0),
                                        (4, dict(DEPTH, ppt=2), 1.0),
                                        (4, dict(DEPTH, bin=4), 1.0),
                                        (4, dict(DEPTH, early_out=2), 1.0),
                                        (4, DEPTH, -1.0), (4, DEPTH, float("inf"))])
def test_bad_entries_are_refused(rz, tmp_path, k, depth, ms):
    with pytest.raises(rz.RzError) as ei:
        rz.tune_cache_store(str(tmp_path / "c.txt"), KEY, k, depth, ACCUM, ms)
    assert ei.value.code == rz.RZ_EINVAL


def test_unwritable_path_reports_io(rz, tmp_path):
    with pytest.raises(rz.RzError) as ei:
        rz.tune_cache_store(str(tmp_path / "no" / "such" / "dir" / "c.txt"), KEY, 4, DEPTH,
                            ACCUM, 1.0)
    assert ei.value.code == rz.RZ_EIO


def test_concurrent_writers_keep_every_entry(rz, tmp_path):
    """Writers of one process are serialised: every key stored by 8 threads
    is in the file afterwards, and the file always parses."""
    path = str(tmp_path / "c.txt")
    errors = []

    def writer(t):
        try:
            for i in range(25):
                rz.tune_cache_store(path, f"gfx950 n{t} px{i} v64 hq4 ordered", 1 + (i % 8),
                                    DEPTH, ACCUM, float(t * 100 + i))
                assert rz.tune_cache_lookup(path, f"gfx950 n{t} px{i} v64 hq4 ordered")
        except Exception as e:  # noqa: BLE001  (reported below)
            errors.append(e)

    th = [threading.Thread(target=writer, args=(t,)) for t in range(8)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors
    for t in range(8):
        for i in range(25):
            e = rz.tune_cache_lookup(path, f"gfx950 n{t} px{i} v64 hq4 ordered")
            assert e["ms"] == float(t * 100 + i) and e["views_per_group"] == 1 + (i % 8)


# ---- order class --------------------------------------------------------

def order_rule(x, y, z):
    """The classifier's rule written out with numpy: three windows of up to
    4096 consecutive points (start, middle, end); a window is ordered when the
    median distance between consecutive finite points is at most 1/16 of the
    diagonal of its finite points' bounding box; the majority of windows with
    at least 16 such pairs decides, ties and no evidence giving shuffled."""
    n = len(x)
    m = min(n, 4096)
    votes = []
    for s in (0, (n - m) // 2, n - m):
        p = np.stack([x[s:s + m], y[s:s + m], z[s:s + m]], 1).astype(np.float64)
        fin = np.isfinite(p).all(1)
        pair = fin[1:] & fin[:-1]
        d = np.sqrt(((p[1:] - p[:-1]) ** 2).sum(1))[pair]
        if d.size < 16:
            continue
        q = p[fin]
        diag = np.sqrt(((q.max(0) - q.min(0)) ** 2).sum())
        med = np.partition(d, d.size // 2)[d.size // 2]
        votes.append(med * 16.0 <= diag)
    return "ordered" if votes and 2 * sum(votes) > len(votes) else "shuffled"


def test_order_class_of_the_generators(rz):
    c = gen.terrain(300_000, 4)
    assert rz.order_class(c.x, c.y, c.z) == "ordered"          # Morton order
    perm = np.random.default_rng(2).permutation(c.n)
    assert rz.order_class(c.x[perm], c.y[perm], c.z[perm]) == "shuffled"
    # a scan-line grid: consecutive points one step apart
    gx, gy = np.meshgrid(np.arange(500, dtype=np.float32), np.arange(400, dtype=np.float32))
    gz = np.zeros_like(gx)
    assert rz.order_class(gx.ravel(), gy.ravel(), gz.ravel()) == "ordered"


@pytest.mark.parametrize("seed", range(12))
def test_order_class_matches_the_rule(rz, seed):
    """Random mixes of ordered runs, shuffled runs, duplicates and NaNs: the
    library's class equals the rule's on every case."""
    rng = np.random.default_rng(seed)
    n = int(rng.choice([0, 1, 15, 17, 100, 4096, 5000, 20000]))
    t = np.cumsum(rng.exponential(1.0, n)).astype(np.float32)
    x, y, z = t.copy(), (0.5 * t).copy(), np.zeros(n, np.float32)
    if n and rng.random() < 0.6:   # shuffle a random part
        a, b = sorted(rng.integers(0, n, 2))
        p = rng.permutation(np.arange(a, b))
        x[a:b], y[a:b] = x[p], y[p]
    if n and rng.random() < 0.4:
        x[rng.integers(0, n, max(1, n // 7))] = np.nan
    if n and rng.random() < 0.2:
        x[:], y[:] = 1.0, 2.0      # every point the same
    got = rz.order_class(x, y, z)
    assert got == order_rule(x, y, z), (seed, n)


def test_order_class_edge_cases(rz):
    assert rz.order_class(np.zeros(0), np.zeros(0), np.zeros(0)) == "shuffled"
    nan = np.full(5000, np.nan, np.float32)
    assert rz.order_class(nan, nan, nan) == "shuffled"
    with pytest.raises(rz.RzError):
        rz.order_class(np.zeros(3), np.zeros(4), np.zeros(3))
