"""Serving behaviour on the GPU: continuous batching of canonical requests, sampling as part of
a request, the reference cache switch, the stage profile, cancellation and admission."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import dev, empty, host, require_gpu

pytestmark = pytest.mark.gpu


def mixed_problems(n, seed=5):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        L = tuple(int(x) for x in rng.integers(2, 9, 3))
        kind = int(rng.integers(0, 3))
        param = (0.0, 0.5, 1.0)[kind]
        N = tuple(int(2 * rng.integers(30, 70) + 1) for _ in range(3))
        h = float(rng.uniform(0.15, 0.3))
        blk = W.Block(L, (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))
        nd = int(rng.integers(0, 4))
        defects = W.draw_defects(rng, [blk], nd // 2, nd - nd // 2)
        # odd requests keep FP32 factors, so batches mix the two sampling groups
        prec = W.FP32 if i % 2 else W.FP64
        out.append(W.Problem(f"m{i}", kind, param, 24, N, h, [blk], defects, precision=prec))
    return out


def test_batched_results_equal_alone():
    require_gpu()
    import torch
    import paper_1411_1994_amd as L
    probs = mixed_problems(24)
    rng = np.random.default_rng(1)
    pts = [rng.uniform(-np.array(W.half_widths(p)), np.array(W.half_widths(p)), size=(257, 3)) for p in probs]
    alone = []
    with L.Context(0, n_slots=1) as c1:
        c1.set_option(L.OPT_MAX_BATCH, 1)
        for p, x in zip(probs, pts):
            r = c1.submit(p, points=x)
            assert r.wait() == 0
            assert r.stats()["batch"] == 1
            alone.append(r.values.copy())
            r.release()
    with L.Context(0, n_slots=2) as c2:
        c2.set_option(L.OPT_MAX_BATCH, 16)
        xs = [dev(x) for x in pts]
        outs = [empty(len(x), torch.float64) for x in pts]
        reqs = [c2.submit(p, points=x, values=o) for p, x, o in zip(probs, xs, outs)]
        batches = []
        for r in reqs:
            assert r.wait() == 0
            batches.append(r.stats()["batch"])
        for r, o, a in zip(reqs, outs, alone):
            assert np.array_equal(host(o), a)            # bitwise: batch-invariant kernels
            r.release()
        assert max(batches) > 1                           # some requests really were fused
        prof = c2.profile()
        assert prof["shift_sum"]["launches"] < len(probs)
        assert prof["shift_sum"]["bytes"] > 0
        assert prof["sample"]["launches"] < len(probs)          # canonical sampling fused per batch too


def test_completion_sampling_matches_oracle_and_lsum_sample():
    require_gpu()
    import paper_1411_1994_amd as L
    p = mixed_problems(1, seed=9)[0]
    rng = np.random.default_rng(2)
    cells = np.stack([rng.integers(0, n, 200) for n in p.N], axis=1)
    xyz = np.stack([(cells[:, a] - (p.N[a] - 1) // 2) * p.h for a in range(3)], axis=1)
    with L.Context(0) as c:
        r = c.submit(p, points=xyz)
        assert r.wait() == 0
        ref = O.brute_force_points(p, cells)
        assert np.max(np.abs(r.values - ref)) <= 1e-12 * np.max(np.abs(ref))
        assert np.array_equal(r.sample(xyz), r.values)
        r.release()


def test_reference_cache_switch_gives_identical_results():
    require_gpu()
    import paper_1411_1994_amd as L
    probs = mixed_problems(6, seed=3)
    pts = np.array([[0.1, 0.2, 0.3], [-1.0, 2.0, 0.5]])
    res = []
    for cache in (1 << 30, 0):
        with L.Context(0, n_slots=1) as c:
            c.set_option(L.OPT_REF_CACHE_BYTES, cache)
            vals = []
            for p in probs + probs:                        # second pass hits the cache when on
                r = c.submit(p, points=pts)
                assert r.wait() == 0
                vals.append(r.values.copy())
                r.release()
            prof = c.profile()
            res.append((vals, prof["collocate"]["launches"]))
    assert all(np.array_equal(a, b) for a, b in zip(res[0][0], res[1][0]))
    assert res[0][1] < res[1][1] == 2 * len(probs)


def test_cancel_and_release_of_queued_requests():
    require_gpu()
    import paper_1411_1994_amd as L
    big = W.config(2)
    with L.Context(0, n_slots=1) as c:
        c.set_option(L.OPT_MAX_BATCH, 1)
        reqs = [c.submit(big) for _ in range(6)]
        cancelled = 0
        for r in reqs[3:]:
            try:
                r.cancel()
                cancelled += 1
            except L.LsumError as e:
                assert e.code == -9                       # already running
        for r in reqs[:3]:
            assert r.wait() == 0
        for r in reqs[3:]:
            assert r.wait() in (0, -6)
        assert cancelled >= 1
        for r in reqs:
            r.release()


def test_submit_many_fuses_one_batch_and_matches_single_submits():
    require_gpu()
    import paper_1411_1994_amd as L
    probs = mixed_problems(10, seed=21)
    singles = []
    with L.Context(0, n_slots=1) as c:
        c.set_option(L.OPT_MAX_BATCH, 1)
        for p in probs:
            r = c.submit(p)
            assert r.wait() == 0
            singles.append([r.canonical(0), r.stats()["batch"]])
            r.release()
    with L.Context(0, n_slots=1) as c:
        c.set_option(L.OPT_MAX_BATCH, 64)
        reqs = c.submit_many(probs)
        for r, (U, _) in zip(reqs, singles):
            assert r.wait() == 0
            assert r.stats()["batch"] == len(probs)            # the whole set ran as one batch
            got = r.canonical(0)
            assert all(np.array_equal(a, b) for a, b in zip(got, U))
            r.release()
        assert c.profile()["shift_sum"]["launches"] == 1
        # an invalid problem anywhere rejects the whole set and queues nothing
        bad = W.Problem(**{**probs[0].__dict__, "N": (20, 21, 21)})
        with pytest.raises(L.LsumError):
            c.submit_many([probs[1], bad, probs[2]])
        assert c.profile()["shift_sum"]["launches"] == 1


def test_large_batch_shift_sum_equals_small_batch():
    # a batch of >= 1024 (64-cell tile, job) pairs takes 48 nodes per workgroup, a small one
    # splits the nodes over the grid; both add the same terms in the same order per entry
    require_gpu()
    import paper_1411_1994_amd as L
    blk = W.Block((5, 4, 3), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))
    p = W.Problem("big", W.NEWTON, 0.0, 30, (2049, 2047, 2045), 0.02, [blk])
    with L.Context(0, n_slots=1) as c:
        c.set_option(L.OPT_MAX_BATCH, 1)
        r = c.submit(p)
        assert r.wait() == 0
        alone = r.canonical(0)
        r.release()
        c.set_option(L.OPT_MAX_BATCH, 64)
        reqs = c.submit_many([p] * 12)                   # 12 x 3 jobs x 32 tiles
        for r in reqs:
            assert r.wait() == 0
            assert r.stats()["batch"] == 12
            assert all(np.array_equal(a, b) for a, b in zip(r.canonical(0), alone))
            r.release()
    ref = O.assembled_canonical(p)[0]
    for a in range(3):
        floor = 1e-13 * np.max(np.abs(ref[a]), axis=1, keepdims=True)
        assert np.all(np.abs(alone[a] - ref[a]) <= 1e-12 * np.abs(ref[a]) + floor)


def test_finish_many_matches_one_by_one():
    # lsum_finish_many waits, reports and releases a set of requests in one call; the values and
    # the reported info are those of waiting on each request
    require_gpu()
    import paper_1411_1994_amd as L
    probs = mixed_problems(6, seed=33)
    rng = np.random.default_rng(4)
    pts = [rng.uniform(-np.array(W.half_widths(p)), np.array(W.half_widths(p)), size=(97, 3)) for p in probs]
    with L.Context(0, n_slots=2) as c:
        one = []
        for p, x in zip(probs, pts):
            r = c.submit(p, points=x)
            assert r.wait() == 0
            one.append((r.values.copy(), r.info().R))
            r.release()
        reqs = c.submit_many(probs, points=pts)
        res = L.finish_many(reqs)
        assert all(r.handle is None for r in reqs)
        for (rc, inf), r, (v, R) in zip(res, reqs, one):
            assert rc == 0 and inf.status == 0 and inf.R == R and inf.t_run_ms >= 0.0
            assert np.array_equal(r.values, v)
        assert L.finish_many([]) == []


def test_request_set_matches_single_submits():
    # a RequestSet (one submit call, one finish call for n requests of one problem) gives each
    # request the values of submitting it alone
    require_gpu()
    import torch
    import paper_1411_1994_amd as L
    p = mixed_problems(1, seed=44)[0]
    rng = np.random.default_rng(8)
    x = rng.uniform(-np.array(W.half_widths(p)), np.array(W.half_widths(p)), size=(301, 3))
    with L.Context(0, n_slots=2) as c:
        r = c.submit(p, points=x)
        assert r.wait() == 0
        alone = r.values.copy()
        r.release()
        xd = dev(x)
        outs = [empty(len(x), torch.float64) for _ in range(5)]
        rs = c.submit_set(L.prepare(p), 5, points=xd, values=outs)
        status, infos = rs.finish()
        assert list(status) == [0] * 5 and all(infos[k].status == 0 for k in range(5))
        for o in outs:
            assert np.array_equal(host(o), alone)


def _served_mix(n):
    """The first n requests of the seeded served mixed workload: rectangular lattices L_l in
    [8, 96], N up to 4097, Newton / Yukawa / Slater, 0..500 vacancies and impurities, eps in
    {1e-4 (FP32 contractions), 1e-6 (FP64)}; every one is an RHOSVD request."""
    return [p for _, p in W.served_stream(n, 1.0)]


def test_served_mix_rhosvd_alone_equals_mix_and_oracle():
    # Eight requests of the served mix (all three kernels, N from 243 to 4097, 59..345 defects,
    # both eps), each run alone (one slot, no batching) and then all together on three slots,
    # where their shift-sums, range bases, per-mode Jacobi SVDs and contractions overlap on the
    # device.  Ranks, certified bounds and values at 64 points are bitwise those of the alone
    # runs (every kernel sums in a fixed order whatever runs beside it), and at sampled points
    # each result is within eps (relative to the largest value) of the oracle's direct sum.
    require_gpu()
    import paper_1411_1994_amd as L
    probs = _served_mix(8)
    assert {p.kind for p in probs} == {0, 1, 2} and {p.eps for p in probs} == {1e-4, 1e-6}
    assert max(max(p.N) for p in probs) == 4097
    rng = np.random.default_rng(55)
    pts = [rng.uniform(-np.array(W.half_widths(p)), np.array(W.half_widths(p)), size=(64, 3)) for p in probs]
    alone = []
    with L.Context(0, n_slots=1) as c1:
        c1.set_option(L.OPT_MAX_BATCH, 1)
        for i, (p, x) in enumerate(zip(probs, pts)):
            print(f"alone {i}: kernel {p.kind} N {p.N} defects {len(p.defects)} eps {p.eps}", flush=True)
            r = c1.submit(p, points=x)
            assert r.wait() == 0, r.stats()
            inf = r.info()
            alone.append((r.values.copy(), tuple(inf.r), inf.bound, inf.norm_A))
            r.release()
    with L.Context(0, n_slots=3) as c3:
        reqs = [c3.submit(p, points=x) for p, x in zip(probs, pts)]
        for i, (r, (v, ranks, bound, nA)) in enumerate(zip(reqs, alone)):
            assert r.wait() == 0, r.stats()
            inf = r.info()
            assert tuple(inf.r) == ranks and inf.bound == bound and inf.norm_A == nA, i
            assert np.array_equal(r.values, v), i
            r.release()
    for i, (p, x) in enumerate(zip(probs, pts)):
        sel = [0, 1, 2]
        ref = O.brute_force_points(p, O.points_to_cells(x[sel], p.h, p.N))
        err = np.max(np.abs(alone[i][0][sel] - ref)) / np.max(np.abs(ref))
        assert err <= p.eps, (i, err)


def test_request_failing_mid_run_leaves_others_unchanged():
    # A request made to fail from the host in the middle of its run: with the Jacobi sweep limit
    # at 1 every side-matrix SVD stops unconverged, so the reduction requests fail with
    # LSUM_E_NOCONV after their shift-sums, side matrices and norms have run (every kernel exits
    # normally), while canonical requests on the other slots complete with the values they have
    # alone.  With the limit restored the same context serves the reduction requests again, with
    # the values they have on a fresh context.
    require_gpu()
    import paper_1411_1994_amd as L
    canon = mixed_problems(6, seed=71)
    red = [p for _, p in W.served_stream(3, 1.0, seed_offset=9, L_range=(6, 14), n_choices=(129, 257),
                                         max_defects=40)]
    rng = np.random.default_rng(72)
    pts = [rng.uniform(-np.array(W.half_widths(p)), np.array(W.half_widths(p)), size=(50, 3))
           for p in canon + red]
    ref = []
    with L.Context(0, n_slots=1) as c1:
        for p, x in zip(canon + red, pts):
            r = c1.submit(p, points=x)
            assert r.wait() == 0
            ref.append(r.values.copy())
            r.release()
    with L.Context(0, n_slots=3) as c:
        c.set_option(L.OPT_JACOBI_MAX_SWEEPS, 1)
        order = [canon[0], red[0], canon[1], canon[2], red[1], canon[3], red[2], canon[4], canon[5]]
        reqs = [c.submit(p, points=pts[(canon + red).index(p)]) for p in order]
        for p, r in zip(order, reqs):
            rc = r.wait()
            k = (canon + red).index(p)
            if p.eps > 0:
                assert rc == -10, (rc, order.index(p), r.stats().get("error"))   # LSUM_E_NOCONV, mid-run
            else:
                assert rc == 0, (rc, order.index(p), r.stats().get("error"))
                assert np.array_equal(r.values, ref[k])
            r.release()
        c.set_option(L.OPT_JACOBI_MAX_SWEEPS, 40)
        for k, p in enumerate(canon + red):
            r = c.submit(p, points=pts[k])
            assert r.wait() == 0
            assert np.array_equal(r.values, ref[k])
            r.release()
        with pytest.raises(L.LsumError):
            c.set_option(L.OPT_JACOBI_MAX_SWEEPS, 0)
