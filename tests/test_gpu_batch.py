"""The persistent batched rounding (one launch for many tensors, Sec. 3.3
applied per tensor, adaptive decisions on the device): parity with the
oracle on small, edge and C4-shaped tensors (including tensors rounded by
teams of several workgroups), results independent of the rest of the batch
(bitwise), and graph capture with replays that recompute every result."""
import math

import numpy as np
import pytest
import torch

import ttgen
from oracle import krp, tt
from gpu_helpers import rel_tensor_diff, say, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = 1e-10     # float64 path vs the float64 oracle, relative to ||X||
TIE = 1e-6      # |est - tau| / tau below which a rank decision may differ


def _check_vs_oracle(x, y, info, tol, ell_block, seed):
    yo, io = krp.round_adaptive(x, tol, ell_block, seed)
    if info["ranks"] != io["ranks"]:
        # an adaptive decision at est ~ tau: both results must meet the bound
        assert io["min_margin"] < TIE, (info["ranks"], io["ranks"], io["min_margin"])
        nx = tt.norm(x)
        assert tt.diff_norm(x, y) <= 1.5 * tol * nx
        assert tt.diff_norm(x, yo) <= 1.5 * tol * nx
        return math.nan
    d = rel_tensor_diff(x, y, yo)
    assert d <= TOL, d
    return d


def _cases():
    return [
        (ttgen.c1(), 1e-8, 42),
        (ttgen.small_random(21, 2, [30, 25], [12]), 1e-6, 5),
        (ttgen.small_random(22, 3, [1, 5, 4], [1, 4]), 1e-6, 6),
        (ttgen.small_random(23, 4, [3, 2, 3, 2], [3, 6, 2]), 1e-8, 7),
        (ttgen.small_random(24, 5, [7, 70, 3, 9, 4], [7, 37, 20, 4]), 1e-4, 8),
    ]


@pytest.mark.parametrize("ell_block", [4, 0])
def test_batch_small_and_edge_shapes_vs_oracle(lib, ell_block):
    cases = _cases()
    say("batch small/edge, ell_block", ell_block)
    plan = lib.BatchPlan([to_dev(x) for x, _, _ in cases], [t for _, t, _ in cases], ell_block,
                         [s for _, _, s in cases])
    plan.launch()
    res = plan.finish()
    for (x, tol, seed), (y, info) in zip(cases, res):
        say("  ranks", info["ranks"])
        _check_vs_oracle(x, to_host(y), info, tol, ell_block, seed)
        assert tt.left_orth_defect(to_host(y)) < 1e-12


def _c4_sample():
    shapes = ttgen.c4_shapes()
    # every 32nd tensor plus the three with the largest cores (rounded by teams)
    sizes = [d * n * r * r for d, n, r in ((s[0], s[1], 3 * s[2]) for s in shapes)]
    big = sorted(range(len(shapes)), key=lambda t: -sizes[t])[:3]
    idx = sorted(set(list(range(0, len(shapes), 32)) + big))
    return idx, [ttgen.c4_one(1004 * 1000 + t, *shapes[t]) for t in idx]


def test_batch_c4_sample_vs_plain_and_oracle(lib):
    idx, xs = _c4_sample()
    devs = [to_dev(x) for x in xs]
    seeds = [42 + t for t in idx]
    plan = lib.BatchPlan(devs, 1e-6, 16, seeds)
    teams = [plan.team(i) for i in range(len(xs))]
    say("C4 sample", idx, "teams", teams)
    assert max(teams) > 1  # the team barriers and row splits are exercised
    plan.launch()
    res = plan.finish()
    for t, x, dv, sd, (y, info) in zip(idx, xs, devs, seeds, res):
        yp, ip = lib.round_adaptive(dv, 1e-6, 16, sd)
        say("  tensor", t, "ranks", info["ranks"][:4], "...")
        assert info["ranks"] == ip["ranks"]
        assert rel_tensor_diff(x, to_host(y), to_host(yp)) <= 1e-12
        assert tt.diff_norm(x, to_host(y)) <= 1e-6 * tt.norm(x)
        # the blocks' final QR after reorthogonalisation is one CholeskyQR pass
        assert tt.left_orth_defect(to_host(y)) < 1e-12
    # the oracle on the tensor with the largest team and two others
    for j in sorted(range(len(xs)), key=lambda j: -teams[j])[:1] + [0, 1]:
        say("  oracle, tensor", idx[j])
        _check_vs_oracle(xs[j], to_host(res[j][0]), res[j][1], 1e-6, 16, seeds[j])


def test_batch_ranks_above_128_vs_oracle(lib):
    """Formal ranks above 128 take the kernel's unstaged paths: the
    contraction of a core with r_k > 128, the sketch and the block updates
    with K > 128, and the next core through the LDS-staged tiles; once
    alone and once in a team of two (threshold lowered for the test)."""
    a = ttgen.small_random(31, 4, 12, [12, 70, 12])
    b = ttgen.small_random(32, 4, 12, [12, 70, 12])
    x = tt.formal_sum([a, b], [1.0, 1e-3])
    assert max(tt.ranks_of(x)) > 128
    say("batch ranks > 128", tt.ranks_of(x))
    prev = lib.batch_team_flops(0.0)
    try:
        for f0 in (1e12, 1e3):
            lib.batch_team_flops(f0)
            plan = lib.BatchPlan([to_dev(x)], 1e-8, 16, [11])
            say("  team", plan.team(0))
            plan.launch()
            (y, info), = plan.finish()
            say("  ranks", info["ranks"])
            _check_vs_oracle(x, to_host(y), info, 1e-8, 16, 11)
            assert tt.left_orth_defect(to_host(y)) < 1e-12
    finally:
        lib.batch_team_flops(prev if prev > 0 else -1.0)


def test_batch_result_independent_of_the_batch(lib):
    """Each tensor's result is bitwise the same alone and in the batch."""
    idx, xs = _c4_sample()
    devs = [to_dev(x) for x in xs]
    seeds = [42 + t for t in idx]
    plan = lib.BatchPlan(devs, 1e-6, 16, seeds)
    plan.launch()
    res = plan.finish()
    for j in [0, len(xs) // 2, len(xs) - 1]:
        alone = lib.BatchPlan([devs[j]], 1e-6, 16, [seeds[j]])
        alone.launch()
        (ya, ia), = alone.finish()
        say("  alone vs mix, tensor", idx[j], "team", alone.team(0))
        assert ia["ranks"] == res[j][1]["ranks"]
        for u, v in zip(ya, res[j][0]):
            assert torch.equal(u, v)


def test_batch_graph_capture_replays(lib):
    """The launch recorded in a graph and replayed three times, with eager
    work between the replays and the outputs overwritten before each: every
    replay reproduces the eager results bitwise."""
    idx, xs = _c4_sample()
    xs, idx = xs[:6], idx[:6]
    devs = [to_dev(x) for x in xs]
    seeds = [42 + t for t in idx]
    plan = lib.BatchPlan(devs, 1e-6, 16, seeds)
    plan.launch()
    ref = [([c.clone() for c in y], info["ranks"]) for y, info in plan.finish()]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        plan.launch()
    torch.cuda.synchronize()
    for rep in range(3):
        for b in plan.bufs:
            for c in b:
                c.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = plan.finish()
        say("  replay", rep, "junk", float(junk) * 0.0)
        for (y, info), (yr, rk) in zip(got, ref):
            assert info["ranks"] == rk
            for u, v in zip(y, yr):
                assert torch.equal(u, v)


def test_batch_block_limits(lib):
    """Sketch blocks are capped by the rank caps (ell_block 65 on C1, whose
    caps are at most 30, is valid); a tensor whose blocks could exceed 64
    columns is refused with TT_EUNSUPPORTED."""
    x = ttgen.c1()
    plan = lib.BatchPlan([to_dev(x)], 1e-8, 65, [1])
    plan.launch()
    (y, info), = plan.finish()
    _check_vs_oracle(x, to_host(y), info, 1e-8, 65, 1)
    wide = ttgen.small_random(31, 3, [100, 100, 5], [90, 5])
    with pytest.raises(lib.TTError) as e:
        lib.BatchPlan([to_dev(wide)], 1e-8, 65, [1])
    assert e.value.status == -6


def test_batch_autotune_sets_the_device_threshold(lib, tmp_path, monkeypatch):
    """The autotuner times every candidate team threshold on the batch,
    makes the fastest the device's and appends it to the cache file; plans
    created afterwards size their teams by it; a cleared value is read back
    from the cache file; results under any threshold agree with the plain
    rounding."""
    idx, xs = _c4_sample()
    devs = [to_dev(x) for x in xs]
    seeds = [42 + t for t in idx]
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("TTR_BATCH_TUNE_CACHE", str(cache))
    try:
        best, times = lib.batch_autotune(devs, 1e-6, 16, seeds, candidates=(1e12, 1e8))
        say("autotune", best, times)
        assert set(times) == {1e12, 1e8} and all(t > 0 for t in times.values())
        assert best == min(times, key=times.get)
        assert lib.batch_team_flops() == best
        key, val = cache.read_text().split("\n")[-2].split()
        assert float(val) == best and key.startswith("gfx")
        # teams follow the device's threshold
        lib.batch_team_flops(1e12)
        one = lib.BatchPlan(devs, 1e-6, 16, seeds)
        assert all(one.team(i) == 1 for i in range(len(xs)))
        lib.batch_team_flops(1e8)
        many = lib.BatchPlan(devs, 1e-6, 16, seeds)
        assert max(many.team(i) for i in range(len(xs))) > 1
        for plan in (one, many):
            plan.launch()
            res = plan.finish()
            for j in (0, len(xs) - 1):
                yp, ip = lib.round_adaptive(devs[j], 1e-6, 16, seeds[j])
                assert res[j][1]["ranks"] == ip["ranks"]
                assert rel_tensor_diff(xs[j], to_host(res[j][0]), to_host(yp)) <= 1e-12
        # cleared: the cache file's entry for this device applies again
        cache.write_text(cache.read_text() + "%s %r\n" % (key, 2.5e9))
        assert lib.batch_team_flops(-1) == 2.5e9
    finally:
        monkeypatch.delenv("TTR_BATCH_TUNE_CACHE")
        lib.batch_team_flops(-1)  # back to the default for the other tests
    assert lib.batch_team_flops() == 3e9
