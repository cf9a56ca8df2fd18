"""The seeded input generators: published SplitMix64 outputs, determinism and
the distributions the workloads promise. CPU only."""

import numpy as np

from paper_2508_04701_amd import datagen as g


def test_splitmix64_published_vector():
    # Reference outputs of SplitMix64 seeded with 1234567 (Vigna's splitmix64.c).
    expect = [6457827717110365317, 3203168211198807973, 9817491932198370423,
              4593380528125082431, 16408922859458223821]
    assert [g.splitmix64_at(1234567, i) for i in range(5)] == expect


def test_same_seed_same_bytes():
    a = g.star_schema(seed=5, n_fact=50_000, n_dim_a=3000, n_dim_b=200, attributes=True)
    b = g.star_schema(seed=5, n_fact=50_000, n_dim_a=3000, n_dim_b=200, attributes=True)
    c = g.star_schema(seed=6, n_fact=50_000, n_dim_a=3000, n_dim_b=200)
    for k in c:
        assert np.array_equal(a[k], b[k])
    assert not np.array_equal(a["date"], c["date"])


def test_prefix_stability():
    # counter-based draws: a longer column extends a shorter one
    a = g.uniform(1, 2, 0, 1000, 1000, np.int32)
    b = g.uniform(1, 2, 0, 1000, 5000, np.int32)
    assert np.array_equal(a, b[:1000])


def test_ranges_and_permutations():
    d = g.star_schema(seed=1, n_fact=200_000, n_dim_a=5000, n_dim_b=300)
    assert d["date"].min() >= 0 and d["date"].max() < 2557
    assert d["price"].min() >= 100 and d["price"].max() < 10_000_000
    assert set(np.unique(d["flag"])) == {0, 1, 2}
    assert d["fk_a"].max() < 5000 and d["fk_b"].max() < 300
    assert np.array_equal(np.sort(d["dim_a_key"]), np.arange(5000))
    assert np.array_equal(np.sort(d["dim_b_key"]), np.arange(300))
    # about 30% of dates fall below 767
    frac = (d["date"] < 767).mean()
    assert abs(frac - 767 / 2557) < 0.01


def test_join_groupby_match_rate():
    d = g.join_groupby()
    assert np.array_equal(np.sort(d["build_key"]), np.arange(65536))
    miss = (d["probe_key"] >= 65536).mean()
    assert abs(miss - (72090 - 65536) / 72090) < 0.002


def test_skewed_keys():
    d = g.skewed(n_build=20_000, n_probe=200_000, n_groups=2000)
    assert len(np.unique(d["build_key"])) == 20_000
    # every probe key is a build key
    assert np.isin(d["probe_key"], d["build_key"]).all()
    # the most frequent key carries about 1/H_N of the probes
    H = float(np.sum(1.0 / np.arange(1, 20_001)))
    top = np.unique(d["probe_key"], return_counts=True)[1].max() / 200_000
    assert abs(top - 1.0 / H) < 0.01
    assert len(np.unique(d["probe_grp"])) <= 2000


def test_batch_shapes():
    shapes = g.batch_shapes()
    assert len(shapes) == 256
    nb = np.array([s["n_build"] for s in shapes])
    npr = np.array([s["n_probe"] for s in shapes])
    ng = np.array([s["n_groups"] for s in shapes])
    assert nb.min() >= 1000 and nb.max() <= 4_000_000
    assert npr.min() >= 10_000 and npr.max() <= 50_000_000
    assert ng.min() >= 8 and np.all(ng <= nb)
    inst = g.batch_instance(7, 3, 2000, 10_000, 50)
    assert np.array_equal(np.sort(inst["build_key"]), np.arange(2000))
    assert abs(np.isin(inst["probe_key"], inst["build_key"]).mean() - 0.9) < 0.02
