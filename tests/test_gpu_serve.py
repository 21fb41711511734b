"""Serving on the GPU: every request's result is the same alone and in the mix
(bitwise: same kernels, same shapes, no atomics on the output path), results match
the oracle, and the budget holds while requests queue and overlap."""
import numpy as np
import pytest

import oracle as O
from paper_2105_01612_amd import workload as wl

pytestmark = pytest.mark.gpu


def test_alone_equals_mix_and_oracle():
    import torch
    from paper_2105_01612_amd.serve import GpuBackend, Request, Server

    sizes = (32, 48, 64)
    host = {n: np.stack([wl.voronoi_field(wl.FieldSpec((n, n, n), grains=max(2, n ** 3 // 16 ** 3),
                                                      sigma_grain=100.0, sigma_noise=5.0, seed=4100 + 7 * n + j),
                                          dtype=np.float32) for j in range(2)]) for n in sizes}
    pools = {n: torch.from_numpy(a).cuda() for n, a in host.items()}
    torch.cuda.synchronize()
    be = GpuBackend(pools, prec="fp32", op="ddo")
    budget = be.slot_bytes(64) + be.slot_bytes(48) + 2 * be.slot_bytes(32)
    arr = wl.poisson_arrivals(40, 4000.0, seed=11)
    ns = wl.request_sizes(40, seed=11, sizes=sizes)
    reqs = [Request(i, int(n), float(t), i % 2) for i, (t, n) in enumerate(zip(arr, ns))]
    mix = {}
    srv = Server(be, budget, max_slots_per_class=2)
    stats = srv.run(reqs, on_complete=lambda r, out: mix.__setitem__(r.rid, out.cpu().numpy().copy()))
    assert stats["completed"] == 40 and srv.peak_used <= budget
    srv.close()
    for r in reqs[:12]:
        alone = {}
        s1 = Server(GpuBackend(pools, prec="fp32", op="ddo"), budget)
        s1.run([Request(r.rid, r.n, 0.0, r.field)],
               on_complete=lambda q, out: alone.__setitem__(q.rid, out.cpu().numpy().copy()))
        s1.close()
        assert np.array_equal(alone[r.rid], mix[r.rid]), r
    for r in reqs[:3]:
        ref, _ = O.project(host[r.n][r.field].astype(np.float64), "ddo")
        w = np.array([1, 1, 1, 2, 2, 2.0]).reshape(6, 1, 1, 1)
        d = mix[r.rid] - ref
        assert np.sqrt(np.sum(w * d * d) / np.sum(w * ref * ref)) <= 1e-5
