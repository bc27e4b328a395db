"""Host logic of the batch planner (no GPU): the population plan gives every
instance about the same device time per generation and keeps the batch's
total number of solutions, in powers of two within the bounds."""
import math

from paper_2603_19163_amd import autotune


def test_plan_equalises_device_time():
    counts = {"1:64": 1500, "1:128": 1500, "2:32": 1000}
    costs = {"1:64": 1.0e-6, "1:128": 1.0e-6, "2:32": 8.0e-6}
    plan = autotune.plan_populations(counts, costs, total=80000)
    # P proportional to 1 / cost: the QAP bucket gets an eighth of the TSP population
    assert plan["1:64"] == plan["1:128"] == 8 * plan["2:32"]
    for p in plan.values():
        assert p >= 1 and (p & (p - 1)) == 0
    total = sum(plan[b] * counts[b] for b in counts)
    assert 80000 / math.sqrt(2) <= total <= 80000 * math.sqrt(2)


def test_plan_rounds_in_log_space_and_clamps():
    counts = {"a": 1, "b": 1}
    assert autotune.plan_populations(counts, {"a": 1.0, "b": 1.0}, total=2 * 2.8) == {"a": 2, "b": 2}
    assert autotune.plan_populations(counts, {"a": 1.0, "b": 1.0}, total=2 * 2.9) == {"a": 4, "b": 4}
    assert autotune.plan_populations(counts, {"a": 1.0, "b": 1e6}, total=1000, p_max=64)["a"] == 64
    assert autotune.plan_populations(counts, {"a": 1.0, "b": 1e6}, total=1000)["b"] == 1


def test_buckets():
    assert autotune.bucket_of(1, 20) == "1:32" and autotune.bucket_of(1, 200) == "1:256"
    assert autotune.bucket_of(2, 40) == "2:64" and autotune.bucket_of(1, 5000) == "1:big"


def test_cache_key_follows_the_kernel_sources(tmp_path, monkeypatch):
    """The measurement cache is keyed on a hash of the HIP sources: a changed
    source gives a different key, an unchanged tree the same one."""
    src = tmp_path / "csrc"
    src.mkdir()
    (src / "a.hip").write_text("kernel one")
    (src / "b.hpp").write_text("header")
    monkeypatch.setattr(autotune, "_HERE", str(tmp_path))
    h1 = autotune.kernel_source_hash()
    assert autotune.kernel_source_hash() == h1
    (src / "a.hip").write_text("kernel two")
    assert autotune.kernel_source_hash() != h1
