"""The allocation-free shift-sum entry point (lsum_shift_sum_noalloc) against lsum_shift_sum, the
entry point whose kernels it shares: two calls in a row, the second with a smaller input, each
bitwise equal to the allocating call and within rounding of the oracle's shift-sum; and the
size limit of its static scratch array."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import empty, host, require_gpu

pytestmark = pytest.mark.gpu

COMB_51_2 = [int(np.sign(x) * np.floor(abs(x) + 0.5)) + 1024 for x in (np.arange(40) - 19.5) * 51.2 / 2]


def _one(ctx, M, N_ref, N_axis, sites, h=0.05, runs=False):
    import torch
    import paper_1411_1994_amd as L
    t, w = L.lsum_nodes(W.NEWTON, 0.0, M, (N_ref, N_ref, N_ref), h)
    R = len(t)
    ldg = 2 * N_ref - 1 + 3
    G = empty(R * ldg, torch.float64)
    ctx.collocate(t, w, N_ref, h, G, ldg)
    ldu = N_axis + 2
    sites = np.array(sites, np.int32)
    U_alloc = empty(R * ldu, torch.float64)
    ctx.shift_sum(R, G, ldg, N_ref, N_axis, sites, U_alloc, ldu)
    U_free = torch.full((R * ldu,), float("nan"), dtype=torch.float64, device="cuda")
    ctx.shift_sum_noalloc(R, G, ldg, N_ref, N_axis, sites, U_free, ldu)
    a = host(U_alloc).reshape(R, ldu)[:, :N_axis]
    b = host(U_free).reshape(R, ldu)[:, :N_axis]
    assert np.array_equal(a, b)
    # and the oracle's sum of the same reference rows (positive terms: any order agrees to
    # (n - 1) unit roundoffs relative; runs of one stride read as differences of two compensated
    # strided sums add at most 5 n u of the row's sum)
    Gh = host(G).reshape(R, ldg)[:, :2 * N_ref - 1]
    ref = O.shift_sum(Gh, sites, N_axis, N_ref)
    n = max(1, len(sites))
    floor = 5 * n * 2.0 ** -53 * np.sum(np.abs(Gh), axis=1, keepdims=True) if runs else 0.0
    assert np.all(np.abs(b - ref) <= 1.2e-16 * n * np.abs(ref) + floor)


def test_noalloc_shift_sum_equals_allocating_call_twice():
    require_gpu()
    import paper_1411_1994_amd as L
    with L.Context(0, n_slots=1) as ctx:
        # five interleaved combs (two window tables of 8- and 7-site combs), rank 41
        print("noalloc call 1: N = 2049, 40 sites, M = 40", flush=True)
        _one(ctx, 40, 2049, 2049, COMB_51_2)
        # smaller: one comb (one table) on a shorter axis, fewer nodes; the scratch keeps the
        # first call's tables, which this call overwrites where it reads them
        print("noalloc call 2: N = 777, 70 sites, M = 20", flush=True)
        _one(ctx, 20, 777, 777, list(range(3, 770, 11)))
        # and sites that form no comb (one term per site on the reference rows)
        print("noalloc call 3: N = 129, 4 sites", flush=True)
        _one(ctx, 16, 129, 129, [48, 59, 69, 80])
        # and snapped sites without a short period (b/h = 1024 / 66): 4 runs of stride 31 on the
        # strided prefix and suffix sums, both tables in the scratch array
        print("noalloc call 4: N = 809, 36 sites in runs of one stride", flush=True)
        x = (np.arange(36) - 17.5) * (1024 / 66)
        _one(ctx, 30, 809, 809, [int(np.sign(v) * np.floor(abs(v) + 0.5)) + 404 for v in x], runs=True)


def test_noalloc_shift_sum_rejects_sizes_beyond_its_scratch():
    torch = require_gpu()
    import paper_1411_1994_amd as L
    # 41 rows of 2 * 400001 - 1 entries need two window tables of 131 MB each, beyond the
    # 64 MiB array: refused on the host before any launch
    N_ref = 400001
    ldg = 2 * N_ref - 1
    sites = np.arange(0, 400001, 10000, dtype=np.int32)   # one comb of 41 sites
    with L.Context(0, n_slots=1) as ctx:
        G = torch.zeros(41 * ldg, dtype=torch.float64, device="cuda")
        U = torch.zeros(41 * N_ref, dtype=torch.float64, device="cuda")
        with pytest.raises(L.LsumError) as e:
            ctx.shift_sum_noalloc(41, G, ldg, N_ref, N_ref, sites, U, N_ref)
        assert e.value.code == -4
