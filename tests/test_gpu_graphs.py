"""Jacobi sweeps replayed from captured HIP graphs against the same sweeps launched kernel by
kernel: the truncated SVDs of the side matrices (Def. def:RHOSVD), and everything computed from
them, are the same bit for bit.  Each request replays its graphs over several sweeps with host
work and synchronisation between the replays, and requests follow each other on one context."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def _problems():
    rng = np.random.default_rng(31)
    blocks = [W.Block((24, 24, 24), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))]
    # side matrices with min(D, N) >= 512: the range basis, then Jacobi on the basis rows
    med = W.Problem("med", W.NEWTON, 0.0, 24, (601, 601, 601), 1.0 / 15, blocks,
                    W.draw_defects(rng, blocks, 40, 30), eps=1e-4)
    # small side matrices: the direct Jacobi on the columns
    sblk = [W.Block((7, 6, 5), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))]
    small = W.Problem("small", W.YUKAWA, 0.5, 20, (129, 129, 129), 0.25, sblk,
                      W.draw_defects(rng, sblk, 9, 6), eps=1e-8)
    return [med, small]


def _run(graphs, problems, block=8):
    import paper_1411_1994_amd as L
    out = []
    with L.Context(0, n_slots=1) as c:
        c.set_option(L.OPT_AUTOTUNE, 0)            # the options below decide
        c.set_option(L.OPT_JACOBI_PERSISTENT, 0)   # graphs apply to the round-by-round launches
        c.set_option(L.OPT_JACOBI_BLOCK, block)
        c.set_option(L.OPT_GRAPHS, graphs)
        for p in problems + problems:          # every problem twice on the same context
            rng = np.random.default_rng(6)
            cells = np.stack([rng.integers(0, n, 16) for n in p.N], axis=1)
            xyz = np.stack([(cells[:, a] - (p.N[a] - 1) // 2) * p.h for a in range(3)], axis=1)
            r = c.submit(p)
            assert r.wait() == 0, r.stats()
            st = r.stats()
            out.append(dict(r=tuple(r.info().r), sweeps=tuple(st["sweeps"]), bound=r.info().bound,
                            sig=[s.copy() for s in r.sigma()], v=r.sample(xyz), cells=cells))
            r.release()
    return out


def test_graph_replayed_sweeps_equal_direct_launches():
    require_gpu()
    probs = _problems()
    a, b = _run(1, probs), _run(0, probs)
    a16, b16 = _run(1, probs, 16), _run(0, probs, 16)
    for k, (x, y) in enumerate(zip(a16, b16)):
        assert x["r"] == y["r"] and x["sweeps"] == y["sweeps"] and x["bound"] == y["bound"], k
        assert np.array_equal(x["v"], y["v"]), k
    for k, (x, y) in enumerate(zip(a, b)):
        assert x["r"] == y["r"] and x["sweeps"] == y["sweeps"] and x["bound"] == y["bound"], k
        for l in range(3):
            assert np.array_equal(x["sig"][l], y["sig"][l]), (k, l)
        assert np.array_equal(x["v"], y["v"]), k
    # the same request twice on one context (graphs captured anew per call) gives the same result
    n = len(probs)
    for k in range(n):
        assert np.array_equal(a[k]["v"], a[k + n]["v"])
    # and the replayed result is the lattice sum within its certified bound
    for k, p in enumerate(probs):
        ref = O.brute_force_points(p, a[k]["cells"])
        assert np.max(np.abs(a[k]["v"] - ref)) <= a[k]["bound"] * (1 + 1e-9) + 1e-12 * np.max(np.abs(ref))


def _run_opts(opts, problems):
    # blocks of 8 columns unless the options say otherwise: the persistent ways need them
    import paper_1411_1994_amd as L
    out = []
    with L.Context(0, n_slots=1) as c:
        c.set_option(L.OPT_AUTOTUNE, 0)
        c.set_option(L.OPT_JACOBI_BLOCK, 8)
        for k, v in opts.items():
            c.set_option(k, v)
        for p in problems:
            rng = np.random.default_rng(6)
            cells = np.stack([rng.integers(0, n, 16) for n in p.N], axis=1)
            xyz = np.stack([(cells[:, a] - (p.N[a] - 1) // 2) * p.h for a in range(3)], axis=1)
            r = c.submit(p)
            assert r.wait() == 0, r.stats()
            st = r.stats()
            out.append(dict(r=tuple(r.info().r), sweeps=tuple(st["sweeps"]), bound=r.info().bound, st=st,
                            sig=[s.copy() for s in r.sigma()], v=r.sample(xyz), cells=cells))
            r.release()
    return out


def test_persistent_sweeps_equal_round_by_round_launches():
    # one launch per sweep (rounds ordered by per-block counters) against the round-by-round
    # launches, directly and from graphs: bit for bit the same
    require_gpu()
    import paper_1411_1994_amd as L
    probs = _problems()
    per = _run_opts({L.OPT_JACOBI_PERSISTENT: 1}, probs)
    per4 = _run_opts({L.OPT_JACOBI_PERSISTENT: 2}, probs)
    direct = _run_opts({L.OPT_JACOBI_PERSISTENT: 0, L.OPT_GRAPHS: 0}, probs)
    graph = _run_opts({L.OPT_JACOBI_PERSISTENT: 0, L.OPT_GRAPHS: 1}, probs)
    for k in range(len(probs)):
        for pp in (per, per4):
            assert sum(pp[k]["st"]["jacobi_persistent"]) > 0 and sum(pp[k]["st"]["jacobi_aborted"]) == 0, pp[k]["st"]
        assert sum(direct[k]["st"]["jacobi_persistent"]) == 0
        for other in (direct, graph, per4):
            x, y = per[k], other[k]
            assert x["r"] == y["r"] and x["sweeps"] == y["sweeps"] and x["bound"] == y["bound"], k
            for l in range(3):
                assert np.array_equal(x["sig"][l], y["sig"][l]), (k, l)
            assert np.array_equal(x["v"], y["v"]), k


def test_persistent_sweep_abort_falls_back_to_round_launches():
    # a wait bound of 0 forces the persistent sweeps to abort at their first wait (set from the
    # host; every kernel exits normally).  An aborted sweep wrote only the other buffer, so it runs
    # again round by round from the rows before it: the result is bit for bit that of round-by-
    # round launches throughout, and within its certified bound of the oracle's direct sum
    require_gpu()
    import paper_1411_1994_amd as L
    p = _problems()[0]
    ref = _run_opts({L.OPT_JACOBI_PERSISTENT: 0}, [p])[0]
    for variant in (1, 2):
        got = _run_opts({L.OPT_JACOBI_PERSISTENT: variant, L.OPT_JACOBI_WAIT_US: 0}, [p])[0]
        assert sum(got["st"]["jacobi_aborted"]) >= 1, got["st"]
        assert got["r"] == ref["r"] and got["sweeps"] == ref["sweeps"] and got["bound"] == ref["bound"]
        for l in range(3):
            assert np.array_equal(got["sig"][l], ref["sig"][l]), l
        assert np.array_equal(got["v"], ref["v"])
    nA = ref["st"]["norm_A"]
    assert ref["bound"] <= p.eps * nA * (1 + 1e-12)
    oracle_ref = O.brute_force_points(p, ref["cells"])
    assert np.max(np.abs(ref["v"] - oracle_ref)) <= p.eps * nA


def test_autotuned_sweeps_equal_fixed_ones_and_decisions_persist(tmp_path):
    # the autotuner times the three ways of launching a sweep on the first sweep of each shape
    # bucket and keeps the fastest; results are bit for bit those of a fixed way, and a second
    # context reads the decisions back from the tuning file instead of timing again
    require_gpu()
    import paper_1411_1994_amd as L
    probs = _problems()
    fixed = _run_opts({L.OPT_JACOBI_PERSISTENT: 0}, probs)
    path = str(tmp_path / "tune.txt")
    tuned = []
    for round_ in range(2):
        with L.Context(0, n_slots=1) as c:
            c.set_option(L.OPT_AUTOTUNE, 1)
            c.set_option(L.OPT_JACOBI_BLOCK, 8)   # all four ways (the persistent ones need 8)
            c.tune_file(path)
            for p in probs:
                r = c.submit(p)
                assert r.wait() == 0, r.stats()
                st = r.stats()
                tuned.append(sum(st["jacobi_tuned"]))
                rng = np.random.default_rng(6)
                cells = np.stack([rng.integers(0, n, 16) for n in p.N], axis=1)
                xyz = np.stack([(cells[:, a] - (p.N[a] - 1) // 2) * p.h for a in range(3)], axis=1)
                k = probs.index(p)
                assert np.array_equal(r.sample(xyz), fixed[k]["v"]), k
                assert tuple(st["sweeps"]) == fixed[k]["sweeps"]
                r.release()
            dec = c.tuning()
        assert dec["enabled"] == 1 and any(key.startswith("jacobi/") for key in dec["decisions"]), dec
        for v in dec["decisions"].values():
            assert 0 <= v["choice"] < len(v["ms"]) and v["ms"][v["choice"]] >= 0
    n = len(probs)
    assert sum(tuned[:n]) >= 1          # the first context timed the ways
    assert sum(tuned[n:]) == 0          # the second read the file


@pytest.mark.parametrize("block", [16, 32])
def test_wide_blocks_graphs_equal_direct_and_match_8_column_blocks(block):
    # Jacobi on blocks of 16 or 32 columns: graph replay equals direct launches bit for bit;
    # against blocks of 8 the ranks agree (or sit at a threshold within rounding), both bounds
    # are certified, and both results are within their bound of the oracle's direct sum
    require_gpu()
    import paper_1411_1994_amd as L
    probs = _problems()
    b16d = _run_opts({L.OPT_JACOBI_BLOCK: block, L.OPT_GRAPHS: 0}, probs)
    b16g = _run_opts({L.OPT_JACOBI_BLOCK: block, L.OPT_GRAPHS: 1}, probs)
    b8 = _run_opts({L.OPT_JACOBI_BLOCK: 8}, probs)
    for k, p in enumerate(probs):
        x, y, z = b16d[k], b16g[k], b8[k]
        assert x["r"] == y["r"] and x["sweeps"] == y["sweeps"] and x["bound"] == y["bound"], k
        for l in range(3):
            assert np.array_equal(x["sig"][l], y["sig"][l]), (k, l)
        assert np.array_equal(x["v"], y["v"]), k
        assert all(abs(a - b) <= 1 for a, b in zip(x["r"], z["r"])), (x["r"], z["r"])
        nA = x["st"]["norm_A"]
        ref = O.brute_force_points(p, x["cells"])
        for o in (x, z):
            assert o["bound"] <= p.eps * nA * (1 + 1e-12)
            assert np.max(np.abs(o["v"] - ref)) <= o["bound"] * (1 + 1e-9) + 1e-12 * np.max(np.abs(ref))
        for l in range(3):
            n = min(len(x["sig"][l]), len(z["sig"][l]), min(x["r"][l], z["r"][l]))
            assert np.allclose(x["sig"][l][:n], z["sig"][l][:n], rtol=1e-10, atol=1e-12 * z["sig"][l][0])


@pytest.mark.parametrize("block", [16, 32])
def test_skipped_rotations_match_every_rotation_applied(block):
    # wide-block pair solves leave out rotations below a tenth of the sweep tolerance (and skip
    # steps with none left); with every rotation above the rounding floor applied instead, the
    # certified ranks agree (or sit at a threshold within rounding), both bounds are certified
    # and both results are within their bound of the oracle's direct sum
    require_gpu()
    import paper_1411_1994_amd as L
    probs = _problems()
    on = _run_opts({L.OPT_JACOBI_BLOCK: block, L.OPT_JACOBI_SKIP: 1}, probs)
    off = _run_opts({L.OPT_JACOBI_BLOCK: block, L.OPT_JACOBI_SKIP: 0}, probs)
    for k, p in enumerate(probs):
        x, z = on[k], off[k]
        assert all(abs(a - b) <= 1 for a, b in zip(x["r"], z["r"])), (x["r"], z["r"])
        nA = x["st"]["norm_A"]
        ref = O.brute_force_points(p, x["cells"])
        for o in (x, z):
            assert o["bound"] <= p.eps * nA * (1 + 1e-12)
            assert np.max(np.abs(o["v"] - ref)) <= o["bound"] * (1 + 1e-9) + 1e-12 * np.max(np.abs(ref))
        for l in range(3):
            n = min(len(x["sig"][l]), len(z["sig"][l]), min(x["r"][l], z["r"][l]))
            assert np.allclose(x["sig"][l][:n], z["sig"][l][:n], rtol=1e-10, atol=1e-12 * z["sig"][l][0])
