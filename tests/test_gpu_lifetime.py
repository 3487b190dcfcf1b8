"""Device memory comes back: dose matrices, plans, batched solves and a
server that builds, evicts and destroys matrices leave the device's free
memory where it was (the library's own allocations are counted by the
device, not by torch's caching allocator)."""
import gc

import numpy as np
import pytest

from gpu_util import banner, to_dev
from workloads import SMALL, TINY, draw_batch_instance, penalty_table

pytestmark = pytest.mark.gpu

SLACK = 64 << 20   # allocator granularity and torch's own caching


def _free():
    import torch
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return torch.cuda.mem_get_info()[0]


def test_no_device_memory_leak():
    from paper_0908_4421_amd.imrt import Context, Dose, Plan, Server
    ctx = Context(0)
    Dose.from_geometry(ctx, TINY).close()   # first use of the library's paths
    before = _free()
    rounds = []
    for rep in range(3):
        for spec, storage in ((SMALL, "f32"), (SMALL, "bf16"), (TINY, "f16")):
            d = Dose.from_geometry(ctx, spec, storage=storage)
            p = Plan(ctx, d)
            p.set_structures(None, 4)
            p.set_penalties(penalty_table(spec))
            x = to_dev(np.ones(d.nb, np.float32))
            p.solve(x, eps=1e-4, alpha=2.0, lambda0=2.0 ** -7, max_iter=20, fixed_iters=True, trials_per_pass=2)
            del p, d, x
        doses = [Dose.from_geometry(ctx, s) for s in (TINY, SMALL)]
        plans = []
        for d, s in zip(doses, (TINY, SMALL)):
            p = Plan(ctx, d)
            p.set_structures(None, 4)
            p.set_penalties(penalty_table(s))
            plans.append(p)
        xs = [to_dev(np.ones(d.nb, np.float32)) for d in doses]
        Plan.solve_batch(plans, xs, eps=1e-4, alpha=2.0, lambda0s=[2.0 ** -7] * 2, max_iter=30, fixed_iters=True)
        del plans, doses, xs
        srv = Server(ctx, budget_bytes=40 << 20, max_live=4)
        specs = [draw_batch_instance(s) for s in (1000, 1001, 1002)] + [TINY]
        tk = [srv.submit(10 + i, sp, penalty_table(sp), max_iter=50, fixed_iters=True) for i, sp in enumerate(specs)]
        for t in tk:
            srv.wait(t)
        srv.close()
        del srv
        after = _free()
        banner(f"round {rep}: free memory change {(after - before) / 2**20:+.1f} MiB")
        rounds.append(after)
    # a one-time cost at most (first launches of each kernel), then no growth
    assert before - rounds[0] <= SLACK
    assert all(abs(r - rounds[0]) <= (4 << 20) for r in rounds[1:])
