"""GPU tests of the batched plan: every job's flags, Y, counts, estimates and
gradient must equal the plain one-job-at-a-time path bit for bit (and the
oracle on a sampled job); graph replays must repeat exactly."""
import numpy as np
import pytest
import torch

import oracle
import paper_2604_17066_amd as R
import workloads as WL

pytestmark = pytest.mark.gpu


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _small_batch(ctx, n_scen=4, graphs=(0, 1, 2), Ns=(20_000, 12_345, 777, 3_001)):
    cfg = WL.configs.batched(n_scen=n_scen, N=1, graphs=graphs, ref_scale=0.05)
    systems = []
    for sysd in cfg["systems"]:
        refs = R.Refs(ctx, sysd["n"], 2, sysd["lower"], sysd["upper"])
        system = R.System(ctx, sysd["graph"])
        systems.append((sysd, refs, system))
    jobs = []
    for k, jd in enumerate(cfg["jobs"]):
        sysd, refs, system = systems[jd["system"]]
        N = Ns[k % len(Ns)]
        jobs.append({"model": R.Model(ctx, jd["p"]), "refs": refs, "system": system,
                     "seed": jd["seed"], "N": N, "grad": k % 3 != 2,
                     "buffers": R.Buffers(ctx, sysd["n"], 2, N), "sys": sysd, "p": jd["p"]})
    return jobs, systems


def _plain(ctx, jb):
    b = R.Buffers(ctx, jb["model"].n, 2, jb["N"])
    est, b = R.stage2(ctx, jb["model"], jb["refs"], jb["system"], jb["N"], jb["seed"],
                      form=R.RSR_POPCOUNT, buffers=b)
    return est, b


@pytest.mark.parametrize("tune", [False, True])
def test_plan_equals_plain(rsr_ctx, tune):
    jobs, systems = _small_batch(rsr_ctx)
    plan = R.Plan(rsr_ctx, jobs, tune=tune)
    plan.run()
    est, grads = plan.results()
    for k, jb in enumerate(jobs):
        pe, pb = _plain(rsr_ctx, jb)
        b = jb["buffers"]
        np.testing.assert_array_equal(_np(b.samples), _np(pb.samples), err_msg=f"job {k}")
        np.testing.assert_array_equal(_np(b.flags), _np(pb.flags), err_msg=f"job {k}")
        np.testing.assert_array_equal(_np(b.Y), _np(pb.Y), err_msg=f"job {k}")
        for key, v in pe.items():
            assert est[k][key] == v or (np.isinf(v) and np.isinf(est[k][key])), (k, key)
        if jb["grad"]:
            np.testing.assert_array_equal(grads[k], _np(pb.G), err_msg=f"job {k}")
    plan.close()


def test_plan_job_against_oracle(rsr_ctx):
    jobs, _ = _small_batch(rsr_ctx, n_scen=2, graphs=(1,), Ns=(9_999,))
    plan = R.Plan(rsr_ctx, jobs, tune=True)
    plan.run()
    est, grads = plan.results()
    jb = jobs[1]
    sysd = jb["sys"]
    x = oracle.sample(jb["p"], jb["seed"], 0, 0, jb["N"])
    fl, _, _ = oracle.classify(sysd["lower"], sysd["upper"], x, mode=0)
    Y, _ = oracle.eval_unknown(sysd["graph"], x, fl)
    cnt = oracle.counts(fl, Y)
    oest = oracle.estimate(cnt)
    np.testing.assert_array_equal(_np(jb["buffers"].flags), fl)
    np.testing.assert_array_equal(_np(jb["buffers"].Y), Y)
    assert est[1]["P"] == oest[3] and est[1]["n_u"] == int(cnt[2])
    c, Gref = oracle.grad(jb["p"], x, Y)
    nz = Gref != 0
    assert np.max(np.abs(grads[1][nz] - Gref[nz]) / np.abs(Gref[nz])) <= 1e-5
    plan.close()


def test_plan_replays_identical(rsr_ctx):
    jobs, _ = _small_batch(rsr_ctx, n_scen=3, graphs=(0, 2))
    plan = R.Plan(rsr_ctx, jobs, tune=False)
    ref = None
    for rep in range(10):
        plan.run()
        est, grads = plan.results()
        snap = ([dict(e) for e in est], [g.copy() for g in grads],
                [_np(jb["buffers"].flags).copy() for jb in jobs])
        # Eager work of the program between replays.
        junk = torch.randn(1 << 16, device="cuda").sum().item()
        assert np.isfinite(junk)
        if ref is None:
            ref = snap
            continue
        for a, b in zip(snap[0], ref[0]):
            assert a == b or all(a[k] == b[k] or (np.isinf(a[k]) and np.isinf(b[k])) for k in a)
        for a, b in zip(snap[1], ref[1]):
            np.testing.assert_array_equal(a, b)
        for a, b in zip(snap[2], ref[2]):
            np.testing.assert_array_equal(a, b)
    plan.close()


def test_plan_inconsistent_segment_uses_precedence(rsr_ctx):
    """Rows that are not valid reference states (a lower row above an upper
    row): the plan must keep Algorithm 1's lower precedence."""
    cfg = WL.configs.tiny(N=10)
    n = cfg["n"]
    lower = WL.bernoulli_rows(40, n, 0.85, seed=1)
    upper = WL.bernoulli_rows(30, n, 0.2, seed=2)
    refs = R.Refs(rsr_ctx, n, 2, lower, upper)
    assert not refs.consistent
    system = R.System(rsr_ctx, cfg["graph"])
    jobs = []
    for k in range(3):
        N = 5_000 + 17 * k
        jobs.append({"model": R.Model(rsr_ctx, cfg["p"]), "refs": refs, "system": system,
                     "seed": 50 + k, "N": N, "buffers": R.Buffers(rsr_ctx, n, 2, N)})
    plan = R.Plan(rsr_ctx, jobs, tune=True)
    plan.run()
    est, _ = plan.results()
    for k, jb in enumerate(jobs):
        x = oracle.sample(cfg["p"], jb["seed"], 0, 0, jb["N"])
        fl, _, _ = oracle.classify(lower, upper, x, mode=0)
        np.testing.assert_array_equal(_np(jb["buffers"].flags), fl)
        Y, _ = oracle.eval_unknown(cfg["graph"], x, fl)
        cnt = oracle.counts(fl, Y)
        assert est[k]["n_L"] == int(cnt[0]) and est[k]["n_u_up"] == int(cnt[4])
    plan.close()


def test_plan_tuning_cache(rsr_ctx, tmp_path):
    """A tuning-cache file: the first plan times every segment and writes one
    entry per segment; a second plan over the same shapes reads them back
    (no timing: it is created much faster) and gives identical results; a
    malformed file, or an entry with a chunk cap outside 0..1024, is
    rejected with RSR_EINVAL."""
    import json
    import time
    path = tmp_path / "tune.json"
    jobs, systems = _small_batch(rsr_ctx, n_scen=2, graphs=(0, 2))
    t0 = time.perf_counter()
    plan = R.Plan(rsr_ctx, jobs, tune=str(path))
    t_tuned = time.perf_counter() - t0
    entries = json.loads(path.read_text())
    assert len(entries) == len(systems)
    for key, e in entries.items():
        assert key.startswith(torch.cuda.get_device_properties(0).gcnArchName)
        assert set(e) == {"choice", "first", "growth", "split", "tail", "chunks", "ms"}
        assert e["chunks"] in (0, 8, 16, 32, 128)
    plan.run()
    est1, g1 = plan.results()
    flags1 = [_np(jb["buffers"].flags).copy() for jb in jobs]
    plan.close()
    t0 = time.perf_counter()
    plan = R.Plan(rsr_ctx, jobs, tune=str(path))
    t_cached = time.perf_counter() - t0
    assert json.loads(path.read_text()) == entries
    plan.run()
    est2, g2 = plan.results()
    plan.close()
    print(f"plan creation: tuned {t_tuned:.3f} s, from the cache {t_cached:.3f} s")
    assert t_cached < t_tuned
    for a, b in zip(est1, est2):
        assert a["P"] == b["P"] and a["n_u"] == b["n_u"]
    for a, b in zip(g1, g2):
        np.testing.assert_array_equal(a, b)
    for jb, f in zip(jobs, flags1):
        np.testing.assert_array_equal(_np(jb["buffers"].flags), f)
    bad = tmp_path / "bad.json"
    bad.write_text('{"x": {"choice": 0}}')
    with pytest.raises(R.RSRError) as ei:
        R.Plan(rsr_ctx, jobs, tune=str(bad))
    assert ei.value.status == R.RSR_EINVAL
    assert bad.read_text() == '{"x": {"choice": 0}}'
    # A chunk cap outside 0..1024 is a malformed entry too.
    for chunks in (1025, -1):
        wrong = {k: dict(e, chunks=chunks) for k, e in entries.items()}
        bad.write_text(json.dumps(wrong))
        with pytest.raises(R.RSRError) as ei:
            R.Plan(rsr_ctx, jobs, tune=str(bad))
        assert ei.value.status == R.RSR_EINVAL, chunks


@pytest.mark.parametrize("choice,tail,first,growth,split,chunks",
                         [(0, 0, 16, 4, 64, 0), (0, 1, 16, 6, 256, 0), (0, 1, 16, 8, 512, 0),
                          (0, 2, 32, 4, 64, 0), (0, 2, 32, 8, 256, 0), (4, 2, 32, 6, 256, 0),
                          (0, 0, 8, 4, 16, 2), (0, 1, 8, 4, 16, 1), (0, 1, 16, 4, 32, None)])
def test_plan_cached_cascade_shapes(rsr_ctx, tmp_path, choice, tail, first, growth, split, chunks):
    """Every cascade a tuning cache can name (popcount rounds, matrix-core
    rounds after round 0, matrix-core rounds from round 0 on, the persistent
    cascade: choice 4; split rounds held to 1 or 2 chunks, or an entry
    without "chunks", as written before the key existed) gives the plain
    path's flags, Y and estimates on uneven jobs sharing a launch, on two
    runs of the plan."""
    import json
    path = tmp_path / "tune.json"
    jobs, systems = _small_batch(rsr_ctx, n_scen=2, graphs=(1, 3), Ns=(20_000, 3_001, 777))
    R.Plan(rsr_ctx, jobs, tune=str(path)).close()
    entries = json.loads(path.read_text())
    for e in entries.values():
        e.update(choice=choice, first=first, growth=growth, split=split, tail=tail)
        if chunks is None:
            del e["chunks"]
        else:
            e["chunks"] = chunks
    path.write_text(json.dumps(entries))
    plan = R.Plan(rsr_ctx, jobs, tune=str(path))
    for rep in range(2):
        for jb in jobs:
            jb["buffers"].flags.fill_(7)
        torch.cuda.synchronize()
        plan.run()
        est, _ = plan.results()
        for k, jb in enumerate(jobs):
            pe, pb = _plain(rsr_ctx, jb)
            b = jb["buffers"]
            np.testing.assert_array_equal(_np(b.flags), _np(pb.flags), err_msg=f"job {k} run {rep}")
            np.testing.assert_array_equal(_np(b.Y), _np(pb.Y), err_msg=f"job {k} run {rep}")
            assert est[k]["P"] == pe["P"] and est[k]["n_u"] == pe["n_u"], (k, rep)
    plan.close()


def test_plan_tuning_on_a_job_prefix(rsr_ctx, tmp_path):
    """A segment of six jobs of 1e6 samples: tuning times its candidates on
    the first five (the first jobs reaching 2^22 samples) and stores a
    positive time for the segment; the tuned plan gives the plain path's
    flags, Y and estimates for every job, the one tuning did not time
    included."""
    import json
    path = tmp_path / "tune.json"
    jobs, systems = _small_batch(rsr_ctx, n_scen=6, graphs=(1,), Ns=(1_000_000,))
    plan = R.Plan(rsr_ctx, jobs, tune=str(path))
    entries = json.loads(path.read_text())
    assert len(entries) == 1 and all(e["ms"] > 0 for e in entries.values())
    plan.run()
    est, _ = plan.results()
    for k, jb in enumerate(jobs):
        pe, pb = _plain(rsr_ctx, jb)
        b = jb["buffers"]
        np.testing.assert_array_equal(_np(b.flags), _np(pb.flags), err_msg=f"job {k}")
        np.testing.assert_array_equal(_np(b.Y), _np(pb.Y), err_msg=f"job {k}")
        assert est[k]["P"] == pe["P"] and est[k]["n_u"] == pe["n_u"], k
    plan.close()


def test_plan_persistent_timeout_is_reported(rsr_ctx, tmp_path):
    """A plan whose segments run the persistent cascade (choice 4 from a
    tuning cache) reports a barrier time-out from rsr_plan_results as
    RSR_EHIP: the limit is a launch argument, so it is forced to zero while
    the plan is recorded.  A plan recorded with the default limit gives the
    plain path's flags."""
    import json
    from paper_2604_17066_amd import _abi as A
    path = tmp_path / "tune.json"
    jobs, systems = _small_batch(rsr_ctx, n_scen=2, graphs=(3,), Ns=(60_000, 30_001))
    R.Plan(rsr_ctx, jobs, tune=str(path)).close()
    entries = json.loads(path.read_text())
    for e in entries.values():
        e.update(choice=4, first=32, growth=6, split=256, tail=2)
    path.write_text(json.dumps(entries))
    lib = A.lib()
    try:
        assert lib.rsr_debug_barrier_timeout(0) == A.RSR_OK
        plan = R.Plan(rsr_ctx, jobs, tune=str(path))
        plan.run()
        with pytest.raises(R.RSRError) as ei:
            plan.results()
        assert ei.value.status == A.RSR_EHIP
        plan.close()
    finally:
        lib.rsr_debug_barrier_timeout(-1)
    plan = R.Plan(rsr_ctx, jobs, tune=str(path))
    plan.run()
    est, _ = plan.results()
    for k, jb in enumerate(jobs):
        pe, pb = _plain(rsr_ctx, jb)
        np.testing.assert_array_equal(_np(jb["buffers"].flags), _np(pb.flags), err_msg=f"job {k}")
        assert est[k]["P"] == pe["P"], k
    plan.close()
