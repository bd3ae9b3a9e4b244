"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/siting.h declares, validates arguments before any
launch, and its host-only layout/order helpers agree with the oracle."""
import os
import re

import numpy as np
import pytest

import paper_2006_16783_amd as S
from paper_2006_16783_amd import _lib as L
from synth import uniform_observers

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_every_declared_symbol_is_exported_and_bound():
    hdr = open(os.path.join(ROOT, "include", "siting.h")).read()
    declared = set(re.findall(r"\b(siting_\w+)\s*\(", hdr))
    assert declared, "no declarations parsed"
    lib = L.lib()
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert declared == set(L.EXPORTED)
    assert S.siting_abi_version() == 1


def test_every_source_keeps_the_mandatory_device_flags():
    """Per-source scheduler flags only add to the common ones: every HIP source
    is built for gfx950 at -O3 without packed-FP32 instructions, and extra
    LLVM options reach the device pass only."""
    from paper_2006_16783_amd import build as B
    srcs = [os.path.basename(p) for p in B.sources()]
    assert "vix.hip" in srcs and set(B.FILE_FLAGS) <= set(srcs)
    for name in srcs:
        f = B.flags_of(name)
        assert f[:len(B.HIPCC_FLAGS)] == B.HIPCC_FLAGS
        i = f.index("-packed-fp32-ops")
        assert f[i - 3:i] == ["-Xclang", "-target-feature", "-Xclang"]
        assert "-O3" in f and any(x.startswith("--offload-arch=gfx950") for x in f)
        extra = f[len(B.HIPCC_FLAGS):]
        for j, x in enumerate(extra):
            if x.startswith("-mllvm="):
                assert j > 0 and extra[j - 1] == "-Xarch_device", (name, extra)


def test_validation_errors_before_launch():
    lib = L.lib()
    assert lib.siting_vix(None, 10, 10, 10, 5, 1, 1, 4, 0, None, None) == -1
    assert "NULL" in L.last_error()
    fake = 0x1000  # never dereferenced: validation fails first
    assert lib.siting_vix(fake, 1, 10, 10, 5, 1, 1, 4, 0, fake, None) == -1
    assert lib.siting_vix(fake, 10, 10, 9, 5, 1, 1, 4, 0, fake, None) == -1
    assert lib.siting_vix(fake, 10, 10, 10, 0, 1, 1, 4, 0, fake, None) == -1
    assert lib.siting_vix(fake, 10, 10, 10, 5, -1, 1, 4, 0, fake, None) == -1
    assert lib.siting_vix(fake, 10, 10, 10, 5, 1, 1, 0, 0, fake, None) == -1
    assert lib.siting_vix(fake, 10, 10, 10, 5, 1, 1, 256, 0, fake, None) == -1
    assert lib.siting_findmax(fake, 2, 1, fake, 10, 10, 10, 2, 2, 3, fake, None) == -1
    assert lib.siting_findmax(fake, 0, 1, fake, 10, 10, 10, 11, 2, 3, fake, None) == -1
    assert lib.siting_findmax(fake, 0, 2, fake, 10, 10, 10, 2, 2, 3, fake, None) == -1
    assert lib.siting_findmax(fake, 0, 1, fake, 10, 10, 10, 2, 2, 33, fake, None) == -2
    # viewshed: missing workspace, bad sink, bad schedule
    assert lib.siting_viewshed_batch(fake, 10, 10, 10, fake, 3, fake, None, 5, None, 0,
                                     fake, None, None, None, 0, None) == -4
    assert lib.siting_viewshed_batch(fake, 10, 10, 10, fake, 3, fake, None, 5, None, 7,
                                     fake, None, None, fake, 256, None) == -1
    bad = L.Schedule(0, 1, 0, 0)
    import ctypes
    assert lib.siting_viewshed_batch(fake, 10, 10, 10, fake, 3, fake, None, 5, ctypes.byref(bad),
                                     0, fake, None, None, fake, 256, None) == -1
    assert "waves" in L.last_error()
    # greedy: workspace too small
    assert lib.siting_greedy(fake, fake, fake, 5, 10, 10, 3, 100, fake, fake, fake, fake,
                             fake, 8, None) == -4
    assert lib.siting_greedy(fake, fake, fake, 0, 10, 10, 3, 100, fake, fake, fake, fake,
                             fake, 1 << 20, None) == -1
    assert lib.siting_greedy_workspace_size(100) >= 100 * 12
    # intervisible greedy: same checks, the larger workspace
    assert lib.siting_greedy_intervisible(fake, fake, fake, 5, 10, 10, 3, 100, fake, fake, fake,
                                          fake, fake, 8, None) == -4
    assert lib.siting_greedy_intervisible(fake, fake, fake, 0, 10, 10, 3, 100, fake, fake, fake,
                                          fake, fake, 1 << 20, None) == -1
    assert lib.siting_greedy_workspace_size(100) >= 100 * 32
    # allocation-free greedy: the same argument checks, and a candidate count
    # above its static workspace is rejected before anything is enqueued
    assert lib.siting_greedy_noalloc(fake, fake, fake, 0, 10, 10, 3, 100, fake, fake, fake,
                                     fake, None) == -1
    assert lib.siting_greedy_noalloc(fake, fake, fake, 5, 10, 10, 3, 100, fake, None, None,
                                     fake, None) == -1
    assert lib.siting_greedy_noalloc(fake, fake, fake, L.SITING_GREEDY_NOALLOC_MAX_N + 1, 10,
                                     10, 3, 100, fake, fake, fake, fake, None) == -2
    assert "maximum" in L.last_error()
    # visibility index: negative count, NULL pointers; nothing to do for n = 0
    assert lib.siting_visibility_index(fake, fake, -1, fake, None) == -1
    assert lib.siting_visibility_index(None, fake, 5, fake, None) == -1
    assert lib.siting_visibility_index(None, None, 0, None, None) == 0
    # the counting VIX variant needs its stats buffer
    assert lib.siting_vix_stats(fake, 10, 10, 10, 5, 1, 1, 4, 0, fake, None, None) == -1


def test_layout_matches_oracle_and_rejects_bad_observers(orc):
    for (nr, nc, seed) in [(100, 130, 1), (64, 64, 2), (7, 300, 3)]:
        obs = uniform_observers(nr, nc, 50, seed, roi=(1, 90), height=(0, 30))
        assert (S.siting_viewshed_layout(obs, nr, nc) == orc.layout(obs, nr, nc)).all()
    obs = uniform_observers(50, 50, 5, 1, roi=(1, 10))
    bad = obs.copy()
    bad["x"][2] = 50
    with pytest.raises(S.SitingError):
        S.siting_viewshed_layout(bad, 50, 50)
    bad = obs.copy()
    bad["roi"][0] = 0
    with pytest.raises(S.SitingError):
        S.siting_viewshed_layout(bad, 50, 50)
    bad = obs.copy()
    bad["h_r"][1] = -3
    with pytest.raises(S.SitingError):
        S.siting_viewshed_layout(bad, 50, 50)


def test_order_is_longest_first_permutation():
    obs = uniform_observers(500, 500, 300, 4, roi=(50, 400))
    order = S.siting_viewshed_order(obs)
    assert sorted(order.tolist()) == list(range(300))
    r = obs["roi"][order]
    assert (np.diff(r) <= 0).all()


def test_autotune_candidates_bit_identical_contract():
    c = S.siting_autotune_candidates(100)
    assert len(c) >= 2
    assert any(s.stage_rmax == 100 for s in c) and any(s.stage_rmax == 0 for s in c)
    big = S.siting_autotune_candidates(400)
    assert all(0 <= s.stage_rmax <= 400 for s in big)
    assert any(0 < s.stage_rmax < 400 for s in big)


def test_schedule_cache_round_trip(tmp_path):
    # host logic of the JSON schedule cache, with a stand-in tuner (no GPU)
    import torch
    from paper_2006_16783_amd import schedule_cache as SC
    from paper_2006_16783_amd import Schedule
    calls = []

    def tune(z, obs, off, rmax, bm, order_dev=None):
        calls.append(rmax)
        s = Schedule()
        s.waves, s.groups_per_cu, s.stage_rmax = 8, 3, rmax
        return s, [1.5, 2.5]

    z = torch.zeros((300, 200), dtype=torch.int16)
    obs = torch.zeros((100, 5), dtype=torch.int32)
    path = str(tmp_path / "sched" / "cache.json")
    s1, hit1 = SC.autotune_cached(z, obs, None, 90, None, path, tune=tune)
    s2, hit2 = SC.autotune_cached(z, obs, None, 90, None, path, tune=tune)
    assert (hit1, hit2) == (False, True) and calls == [90]
    assert s1.as_tuple() == s2.as_tuple() == (8, 3, 90, 0)
    # another batch bucket or ROI maximum is tuned again
    SC.autotune_cached(z, torch.zeros((300, 5), dtype=torch.int32), None, 90, None, path, tune=tune)
    SC.autotune_cached(z, obs, None, 120, None, path, tune=tune)
    assert calls == [90, 90, 120]
    assert len(SC.load(path)) == 3
    # 100 and 128 observers share a bucket; a corrupt file reads as empty
    assert SC.cache_key("d", 90, 100, 1, 1) == SC.cache_key("d", 90, 128, 1, 1)
    assert SC.cache_key("d", 90, 129, 1, 1) != SC.cache_key("d", 90, 128, 1, 1)
    open(path, "w").write("{not json")
    assert SC.load(path) == {}


def test_ray_step_counts_match_brute_force():
    # the closed-form per-ray step count against stepping every ray
    from paper_2006_16783_amd import pipeline as P

    def brute(eu, ev, R):
        if eu < 1:
            return 0
        tot = 0
        for rho in range(eu + ev):
            du, dv = (eu, rho) if rho <= ev else (eu - (rho - ev), ev)
            n, mn = max(du, dv), min(du, dv)
            for k in range(1, n + 1):
                m = (2 * k * mn + n) // (2 * n)
                if k * k + m * m > R * R:
                    break
                tot += 1
        return tot

    rng = np.random.default_rng(3)
    for _ in range(200):
        R = int(rng.integers(1, 60))
        eu, ev = int(rng.integers(0, R + 1)), int(rng.integers(0, R + 1))
        assert P._quadrant_ray_steps(eu, ev, R) == brute(eu, ev, R), (eu, ev, R)
    for R in (1, 2, 7, 64):
        assert P._quadrant_ray_steps(R, R, R) == brute(R, R, R)


def test_paper_scale_configs():
    # block grids follow G = round(N / floor(R/3)) (Tables 2 and 3)
    import oracle
    from paper_2006_16783_amd import pipeline as P
    for name, (n, R, G) in {"east_32000_r500": (32000, 500, 193),
                            "east_32000_r1000": (32000, 1000, 96),
                            "west_46400_r1000": (46400, 1000, 139)}.items():
        c = P.CONFIGS[name]
        assert (c.n, c.roi, c.grid, c.k, c.h_t, c.h_r) == (n, R, G, 20, 100, 10)
        assert oracle.block_grid(n, R) == G
