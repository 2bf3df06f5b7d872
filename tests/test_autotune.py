"""Autotuner host logic: shape keys, candidate lists, the JSON cache (no
GPU needed; the timing loop itself is exercised by the GPU batch tests)."""
from types import SimpleNamespace

from paper_1411_3691_amd import autotune


def fake_plan(nf, M, n_src, n_snk):
    return SimpleNamespace(snk=SimpleNamespace(nf=tuple(nf)), M=M, n_src=n_src, n_snk=n_snk)


def test_shape_key_depends_on_every_shape_field():
    base = [fake_plan((6, 6), 48, 100, 90), fake_plan((3, 17), 24, 50, 60)]
    k0 = autotune.shape_key(base, [8, 9], "tree")
    assert k0 == autotune.shape_key(list(base), [8, 9], "tree")
    assert k0 != autotune.shape_key(base, [8, 9], "plain")
    assert k0 != autotune.shape_key(base, [8, 10], "tree")
    assert k0 != autotune.shape_key(base[::-1], [9, 8], "tree")
    for change in (dict(nf=(6, 5)), dict(M=96), dict(n_src=101), dict(n_snk=91)):
        args = dict(nf=(6, 6), M=48, n_src=100, n_snk=90)
        args.update(change)
        assert k0 != autotune.shape_key([fake_plan(**args), base[1]], [8, 9], "tree")


def test_candidates_offer_lane_kernel_only_when_every_job_fits():
    uniform = [fake_plan((6, 6), 48, 10, 10), fake_plan((4, 4), 24, 10, 10)]
    uneven = uniform + [fake_plan((3, 5), 24, 10, 10)]
    grid = dict(kernel=["lane", "group"], blocks_per_cu=[1, 2], items_per_tile=[32])
    c1 = autotune.candidates(uniform, grid)
    assert {c["kernel"] for c in c1} == {"lane", "group"} and len(c1) == 4
    c2 = autotune.candidates(uneven, grid)
    assert {c["kernel"] for c in c2} == {"group"} and len(c2) == 2
    # the default grid: the library's kernel choice, three workgroup counts
    assert len(autotune.candidates(uneven)) == 3


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "tune.json")
    assert autotune.load_cache(path) == {}
    autotune.store_cache(path, "k1", {"schedule": {"kernel": "auto"}, "ms": 1.0})
    autotune.store_cache(path, "k2", {"schedule": {"kernel": "group"}, "ms": 2.0})
    data = autotune.load_cache(path)
    assert data["k1"]["schedule"] == {"kernel": "auto"}
    assert data["k2"]["ms"] == 2.0
