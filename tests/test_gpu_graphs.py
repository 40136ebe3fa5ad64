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


def _run(graphs, problems):
    import paper_1411_1994_amd as L
    out = []
    with L.Context(0, n_slots=1) as c:
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
