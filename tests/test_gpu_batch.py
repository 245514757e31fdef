"""GPU: the batched persistent search (one persistent launch for many
stacks, replayed from a captured HIP graph) against the per-stack search
(bit-identical: the ranking is a total order, so no schedule can change the
result) and against the FP64 oracle (protocol B: both read the oracle's
planes rounded to float32).
"""
import sys

import numpy as np
import pytest
import torch

import synth
from tests import parity as P

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def kbm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_03296_amd as kbm
    kbm.lib()
    return kbm


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


# (stack factory, parameter overrides, region): uneven sizes, epoch counts
# 3..32, k 1..8, filter on and off, masked pixels, a start region, an empty
# region and a one-column image.
BATCH = [
    (lambda: synth.make_config(2, size=(300, 200), n_vel=(16, 24)), {}, None),
    (lambda: synth.make_config(1), {}, None),
    (lambda: synth.tiny_stack(21, W=96, H=40, T=10, n_vel=70, max_speed=12.0),
     dict(k=8, min_obs=6), None),
    (lambda: synth.tiny_stack(22, W=130, H=33, T=30, n_vel=45, mask_rate=0.2,
                              max_speed=3.0), dict(k=4, min_obs=10), None),
    (lambda: synth.tiny_stack(23, W=64, H=17, T=32, n_vel=33, max_speed=2.0),
     dict(k=8, sigmag=0, min_obs=1), None),
    (lambda: synth.make_config(2, size=(300, 200), n_vel=(12, 12)),
     dict(k=6), (5, 3, 290, 150)),
    (lambda: synth.tiny_stack(24, W=1, H=23, T=3, n_vel=40, max_speed=4.0),
     dict(k=2, min_obs=1), None),
    (lambda: synth.tiny_stack(25, W=40, H=30, T=17, n_vel=50), dict(k=3),
     (4, 4, 4, 9)),
]


def _params(kbm, st, over, region):
    p = dict(st.params)
    p.update(over)
    reg = region or (0, 0, st.W, st.H)
    sp = kbm.SearchParams(k=p["k"], min_obs=p["min_obs"], sigmag=bool(p["sigmag"]),
                          q_lo=p["q_lo"], q_hi=p["q_hi"], coeff=p["coeff"],
                          n_sigma=p["n_sigma"], region=reg)
    return p, reg, sp


@pytest.fixture(scope="module")
def batch(kbm, oracle_mod):
    """Stacks, their float32 oracle planes on the GPU, and the per-stack
    search results (the reference for bit-identity)."""
    out = []
    for j, (make, over, region) in enumerate(BATCH):
        st = make()
        p, reg, sp = _params(kbm, st, over, region)
        psi, phi = oracle_mod.planes(st.sci, st.var, st.mask, st.psf)
        psi, phi = psi.astype(np.float32), phi.astype(np.float32)
        item = dict(psi=_cuda(psi), phi=_cuda(phi), times=st.times, vels=st.vels,
                    params=sp)
        _say(f"batch stack {j}: W={st.W} H={st.H} T={st.T} V={len(st.vels)} "
             f"k={p['k']} region={reg}")
        plain = kbm.search(item["psi"], item["phi"], st.times, st.vels, sp)
        out.append(dict(st=st, p=p, reg=reg, item=item, plain=plain,
                        psi=psi, phi=phi))
    torch.cuda.synchronize()
    return out


def _equal(a, b):
    for key in ("lh", "flux", "vel_idx", "n_obs", "keep", "lh_raw"):
        if a.get(key) is None and b.get(key) is None:
            continue
        assert torch.equal(a[key], b[key]), key


def _run(kbm, batch, tune):
    items = [b["item"] for b in batch]
    with kbm.BatchedSearch(items, tune=tune) as plan:
        plan.run()
        assert not plan.check(), "dependency wait gave up"
        return plan.results, plan.schedule


def test_batch_matches_per_stack_search(kbm, batch):
    _say("batch: default schedule vs per-stack search")
    items = [b["item"] for b in batch]
    with kbm.BatchedSearch(items) as plan:
        plan.run()
        assert not plan.check(), "dependency wait gave up"
        _say(f"  schedule {plan.schedule}")
        for b, r in zip(batch, plan.results):
            _equal(r, b["plain"])


def test_batch_other_percentiles(kbm):
    """Stacks with other percentile pairs, clipping widths and masked samples
    (the runtime-rank path of the fused filter) give the per-stack search's
    results bit for bit in one persistent launch."""
    _say("batch: other percentile pairs")
    items = []
    for seed, (T, ql, qh, c, ns) in enumerate([(26, 0.16, 0.84, 0.5035, 2.0),
                                              (17, 0.10, 0.90, 0.39, 3.0),
                                              (9, 0.25, 0.75, 0.7413, 1.5)]):
        st = synth.tiny_stack(40 + seed, W=130, H=37, T=T, n_vel=40, max_speed=12.0,
                              mask_rate=0.1)
        psi, phi = kbm.make_planes(torch.from_numpy(st.sci).cuda(),
                                   torch.from_numpy(st.var).cuda(),
                                   torch.from_numpy(st.mask).cuda(), st.psf)
        items.append(dict(psi=psi, phi=phi, times=st.times, vels=st.vels,
                          params=kbm.SearchParams(k=4, min_obs=max(1, T // 2), q_lo=ql,
                                                  q_hi=qh, coeff=c, n_sigma=ns)))
    with kbm.BatchedSearch(items) as plan:
        plan.run()
        assert not plan.check(), "dependency wait gave up"
        for it, r in zip(items, plan.results):
            ref = kbm.search(it["psi"], it["phi"], it["times"], it["vels"], it["params"])
            _equal(r, ref)


def test_batch_protocol_B(kbm, oracle_mod, batch):
    _say("batch: protocol B against the oracle")
    res, _ = _run(kbm, batch, kbm.TUNE_DEFAULT)
    for j, (b, r) in enumerate(zip(batch, res)):
        st, p, reg = b["st"], b["p"], b["reg"]
        ref = oracle_mod.search(b["psi"], b["phi"], st.times, st.vels, region=reg, **p)

        def single(y, x, v, b=b, st=st, p=p, reg=reg):
            o = oracle_mod.search(b["psi"], b["phi"], st.times, st.vels[v:v + 1], k=1,
                                  region=(reg[0] + x, reg[1] + y, reg[0] + x + 1,
                                          reg[1] + y + 1),
                                  **{k: p[k] for k in ("min_obs", "sigmag", "q_lo",
                                                       "q_hi", "coeff", "n_sigma")})
            return float(o["lh"][0, 0, 0])
        stats = P.compare_search(r, ref, single)
        _say(f"  stack {j}: {stats}")


SCHEDULES = [
    dict(vel_block=32, tile_cols=1, tile_rows=1, waves=1, blocks_per_cu=1, sweep=0),
    dict(vel_block=1000, tile_cols=16, tile_rows=64, waves=4, blocks_per_cu=0, sweep=0),
    dict(vel_block=64, tile_cols=2, tile_rows=32, waves=4, blocks_per_cu=2, sweep=0),
    dict(vel_block=96, tile_cols=8, tile_rows=8, waves=1, blocks_per_cu=0, sweep=0),
    # contiguous shares, including a block that 4 waves do not divide evenly
    dict(vel_block=100, tile_cols=2, tile_rows=32, waves=4, blocks_per_cu=0, sweep=1),
    dict(vel_block=1000, tile_cols=4, tile_rows=16, waves=4, blocks_per_cu=3, sweep=1),
    dict(vel_block=64, tile_cols=1, tile_rows=64, waves=1, blocks_per_cu=0, sweep=1),
]


@pytest.mark.parametrize("sched", SCHEDULES, ids=lambda s: "vb%d_%dx%d_w%d_b%d_s%d" % (
    s["vel_block"], s["tile_cols"], s["tile_rows"], s["waves"], s["blocks_per_cu"],
    s["sweep"]))
def test_batch_schedules_identical(kbm, batch, sched):
    _say(f"batch: schedule {sched}")
    res, used = _run(kbm, batch, sched)
    for f in ("vel_block", "tile_cols", "tile_rows", "waves", "sweep"):
        assert used[f] == sched[f]
    for b, r in zip(batch, res):
        _equal(r, b["plain"])


def test_batch_up_to_27_epochs(kbm, batch):
    """A batch of the shorter stacks only, under the default and an explicit
    schedule."""
    _say("batch: stacks with T <= 27 only")
    sub = [b for b in batch if b["st"].T <= 27]
    assert len(sub) >= 4
    for sched in (None, dict(vel_block=64, tile_cols=2, tile_rows=32, waves=4,
                             blocks_per_cu=0)):
        with kbm.BatchedSearch([b["item"] for b in sub],
                               tune=kbm.TUNE_DEFAULT if sched is None else sched) as plan:
            plan.run()
            assert not plan.check()
            for b, r in zip(sub, plan.results):
                _equal(r, b["plain"])


def test_batch_graph_replay_and_refill(kbm, batch):
    _say("batch: graph replays and refilled planes")
    items = [dict(b["item"], psi=b["item"]["psi"].clone(), phi=b["item"]["phi"].clone())
             for b in batch]
    with kbm.BatchedSearch(items) as plan:
        first = None
        for rep in range(3):
            plan.run()
            assert not plan.check()
            snap = [{k: (v.clone() if v is not None else None) for k, v in r.items()}
                    for r in plan.results]
            if first is None:
                first = snap
            else:
                for a, b in zip(snap, first):
                    _equal(a, b)
            # eager work between replays
            junk = torch.randn(1 << 20, device="cuda").sum()
            torch.cuda.synchronize()
            del junk
        # new images of the same geometry: scale psi (L scales with it)
        for it in items:
            it["psi"].mul_(-0.5)
        plan.run()
        assert not plan.check()
        for it, r in zip(items, plan.results):
            ref = kbm.search(it["psi"], it["phi"], it["times"], it["vels"], it["params"])
            _equal(r, ref)


def test_batch_autotune(kbm, batch, tmp_path, monkeypatch):
    """The autotuned schedule gives the per-stack results; its choice is
    written to the cache file and, once the process forgets it, read back
    (same schedule and probe time, no new tuning)."""
    import json
    cache = tmp_path / "kbm" / "autotune.json"
    monkeypatch.setenv("KBM_TUNE_CACHE", str(cache))
    kbm.tune_cache_clear()
    _say("batch: autotuned schedule")
    res, sched = _run(kbm, batch, kbm.TUNE_AUTO)
    _say(f"  tuned {sched}")
    assert sched["vel_block"] >= 32 and sched["waves"] in (1, 4)
    assert sched["blocks_per_cu"] >= 1 and sched["probe_ms"] > 0
    for b, r in zip(batch, res):
        _equal(r, b["plain"])
    stored = json.loads(cache.read_text())
    assert len(stored) == 1
    (key, val), = stored.items()
    L = kbm.lib()
    L.kbm_build_id.restype = __import__("ctypes").c_char_p
    assert key.startswith(L.kbm_build_id().decode() + "|gfx950")
    assert val[0] == sched["vel_block"] and val[5] == sched["sweep"]
    kbm.tune_cache_clear()
    res2, sched2 = _run(kbm, batch, kbm.TUNE_AUTO)
    assert sched2 == sched
    for b, r in zip(batch, res2):
        _equal(r, b["plain"])


def test_search_batched_default_is_persistent(kbm, batch):
    _say("batch: search_batched picks the persistent kernel")
    items = [b["item"] for b in batch]
    res = kbm.search_batched(items)
    torch.cuda.synchronize()
    for b, r in zip(batch, res):
        _equal(r, b["plain"])


def _valid_count(times, vels, W, H, min_obs):
    """Grid trajectories with at least min_obs epochs inside the image
    (brute force over every start pixel)."""
    t = np.asarray(times, np.float64)
    t = t - t.min()
    v = np.asarray(vels, np.float32).astype(np.float64)
    ys, xs = np.mgrid[0:H, 0:W]
    n = 0
    for j in range(v.shape[0]):
        c = np.zeros((H, W), np.int64)
        for ti in t:
            dx, dy = np.floor(v[j, 0] * ti + 0.5), np.floor(v[j, 1] * ti + 0.5)
            c += (xs + dx >= 0) & (xs + dx < W) & (ys + dy >= 0) & (ys + dy < H)
        n += int(np.sum(c >= min_obs))
    return n


def _skip_rule_count(times, vels, W, H, T, min_obs, region):
    """Trajectory-epochs the sweep evaluates, by brute force over every
    (64-pixel row tile, velocity) pair: a pair is skipped when some epoch of
    some lane leaves the image and, at one of the four image edges, fewer
    than min_obs epochs keep some lane of the tile on the inner side of it."""
    x0, y0, x1, y1 = region
    t = np.asarray(times, np.float64)
    t = t - t.min()
    v = np.asarray(vels, np.float32).astype(np.float64)
    dx = np.clip(np.floor(v[:, :1] * t[None, :] + 0.5), -32767, 32767)
    dy = np.clip(np.floor(v[:, 1:] * t[None, :] + 0.5), -32767, 32767)
    n = 0
    for xw in range(x0, x1, 64):
        lanes = min(64, x1 - xw)
        for y in range(y0, y1):
            inside = ((xw + dx.min(1) >= 0) & (xw + 63 + dx.max(1) <= W - 1) &
                      (y + dy.min(1) >= 0) & (y + dy.max(1) <= H - 1))
            edges = np.stack([(xw + dx <= W - 1).sum(1), (xw + 63 + dx >= 0).sum(1),
                              (y + dy <= H - 1).sum(1), (y + dy >= 0).sum(1)])
            skipped = ~inside & (edges.min(0) < min_obs)
            n += lanes * T * int(np.sum(~skipped))
    return n


def test_batch_evaluated_count(kbm):
    """The evaluated trajectory-epoch count equals a brute-force count of the
    skip rule over every (tile, velocity) pair, regions and the min_obs > T
    case included; it is the nominal count when no track can leave the image
    far enough to fall below min_obs, and at least T x the valid
    trajectories otherwise (a skipped pair holds no valid trajectory)."""
    rng = np.random.default_rng(5)
    T, H, W = 9, 40, 150
    times = np.sort(rng.uniform(0, 2, T))
    psi = torch.from_numpy(rng.normal(size=(T, H, W)).astype(np.float32)).cuda()
    phi = torch.ones_like(psi)
    slow = rng.uniform(-3, 3, size=(40, 2)).astype(np.float32)
    fast = np.concatenate([slow, rng.uniform(-60, 60, size=(80, 2)).astype(np.float32)])
    full = (0, 0, W, H)
    cases = ((slow, 1, full), (fast, 6, full), (fast, 2, (7, 3, 140, 31)),
             (fast, 9, (70, 0, 150, 40)), (fast, T + 1, full))
    for vels, min_obs, region in cases:
        item = dict(psi=psi, phi=phi, times=times, vels=vels,
                    params=kbm.SearchParams(k=3, min_obs=min_obs, region=region))
        with kbm.BatchedSearch([item, item]) as plan:
            plan.run()
            assert not plan.check()
            n = plan.evaluated()
        x0, y0, x1, y1 = region
        nominal = 2 * T * (x1 - x0) * (y1 - y0) * len(vels)
        want = 2 * _skip_rule_count(times, vels, W, H, T, min_obs, region)
        print(f"  min_obs {min_obs} region {region}: evaluated {n} of {nominal}")
        assert n == want
        if vels is slow:
            assert n == nominal
        elif region == full and min_obs <= T:
            assert 2 * T * _valid_count(times, vels, W, H, min_obs) <= n < nominal