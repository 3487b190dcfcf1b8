#!/usr/bin/env python3
"""Time-to-plan of the paper-scale phantom on one MI355X.

One step = one plan optimisation with D already resident in HBM: the initial
step size lambda_0 by 50 power iterations, then gradient projection with
Armijo's line search from x = 1 until the relative objective change drops
below 1e-5 (every forward, adjoint, trial, test and update on the GPU).

Prints one JSON line.  --gpus must be 1: the solver runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
KERNEL_SOURCES = ("paper_0908_4421_amd/csrc/kernels.hip", "paper_0908_4421_amd/csrc/imrt_internal.h")
# counter summaries per workload (by phantom name)
TRAFFIC_PROFILES = {
    "prostate_160x104x80_2.5mm_9field": os.path.join(ROOT, "profiles", "hbm_traffic_fwd_adj_prostate_160x104x80.txt"),
    "scenario3_shape_66x54x40_4mm_9field": os.path.join(ROOT, "profiles",
                                                        "hbm_traffic_fwd_adj_scenario3_shape_66x54x40.txt"),
}


# The byte models count the rows that have nonzeros (nr): a voxel no beamlet
# reaches needs no row pointer, structure id or residual in either pass (its
# zero-dose penalty is a constant of the plan), and the wave forward skips
# every run of 16 or more such rows.


def forward_bytes(nr, nb, nnz):
    """Algorithmic bytes of one forward trial pass: CSR (int32 column, float32
    value, int32 row pointer), structure id, residual out, x_k and g_k in."""
    return 8 * nnz + 4 * (nr + 1) + 1 * nr + 4 * nr + 8 * nb


def forward_bytes_c16(nr, nb, nnz):
    """The same when the forward reads 16-bit column indices beside the
    float32 values (float32 matrices with nb <= 65536, the default)."""
    return 6 * nnz + 4 * (nr + 1) + 1 * nr + 4 * nr + 8 * nb


def f32_forward(ctx, nb):
    """(forward layout code of the kernel name, forward bytes model) of a
    float32 matrix with nb beamlets built under the context's options."""
    if ctx.get_option("fwd_wave") and ctx.get_option("fwd_col16") and nb <= 65536:
        return 3, forward_bytes_c16
    return 0, forward_bytes


def adjoint_bytes(nr, nb, nnz):
    """Algorithmic bytes of one adjoint pass: CSC (int32 row, float32 value,
    int32 column pointer), every residual of a row with nonzeros once,
    gradient out."""
    return 8 * nnz + 4 * (nb + 1) + 4 * nr + 4 * nb


def forward_bytes16(nr, nb, nnz):
    """The same with 16-bit storage: 16-bit column index and code, plus the
    beamlet scales."""
    return 4 * nnz + 4 * (nr + 1) + 1 * nr + 4 * nr + 12 * nb


def adjoint_bytes16(nr, nb, nnz):
    """The same with 16-bit storage: int32 row index and 16-bit code, plus the
    beamlet scales."""
    return 6 * nnz + 4 * (nb + 1) + 4 * nr + 8 * nb


def nonempty_rows(dose):
    """Rows of the dose matrix that hold at least one nonzero."""
    import numpy as np

    from paper_0908_4421_amd.imrt import imrt_dose_export
    rp = np.empty(dose.nv + 1, np.int32)
    imrt_dose_export(dose.handle, row_ptr=rp)
    return int(np.count_nonzero(np.diff(rp)))


def timed_plans(ctx, dose, spec, st, args, warmup, steps):
    """Build a plan on `dose`, run `warmup` untimed and `steps` timed plans
    (lambda_0 estimate plus solve each); returns (ms per plan, results, x, plan)."""
    import numpy as np
    import torch

    from paper_0908_4421_amd.imrt import Plan
    from workloads import penalty_table, power_start_vector
    pl = Plan(ctx, dose)
    pl.set_structures(None, 4)
    pl.set_penalties(penalty_table(spec))
    v0 = torch.as_tensor(power_start_vector(dose.nb, spec.seed).astype(np.float32)).cuda()
    x = torch.empty(dose.nb, dtype=torch.float32, device="cuda")

    def step(profile=0):
        lam0, _ = pl.lambda0(v0, st.power_iters)
        x.fill_(st.x0)
        res, _ = pl.solve(x, eps=st.eps, alpha=st.alpha, lambda0=lam0, delta=st.delta,
                          max_iter=st.max_iter, max_backtracks=st.max_backtracks,
                          fixed_iters=st.fixed_iters, trials_per_pass=args.trials_per_pass,
                          profile=profile)
        return lam0, res

    for _ in range(warmup):
        step()
    # the timed plans carry HIP events around every profile_every-th forward
    # and adjoint launch (recorded on the solver's stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [step(args.profile_every) for _ in range(steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) * 1e3 / steps, runs, x, pl


def kernel_table(runs, res, names, nbytes):
    """Mean HIP-event duration of each pass over the timed plans, with its
    algorithmic bytes per launch and the rate against the HBM peak."""
    kern = {}
    for name in ("forward", "adjoint"):
        ms = sum((r.forward_kernel_ms if name == "forward" else r.adjoint_kernel_ms) for _, r in runs) / len(runs)
        n = res.forward_passes if name == "forward" else res.adjoint_passes
        gbs = nbytes[name] / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        # (a name ending in ", " leaves out the last template argument, the
        # matrix streams' cache policy, which the library picks per matrix)
        label = names[name] + "*>" if names[name].endswith(", ") else names[name]
        kern[name] = {"kernel": label, "avg_ms": ms, "launches": n, "bytes_per_launch": nbytes[name],
                      "GB_s": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS, "total_ms": ms * n}
    return kern


def storage_form(ctx, spec, st, args, storage, plan32, res32, ms32):
    """A plan with D stored as 16-bit codes, timed like the float32 plan, and
    its accuracy against float32 D on the same GPU: the dose of its final x
    under D~ and under D, and G of that x under D against the float32 plan's
    final G."""
    import torch

    from paper_0908_4421_amd.imrt import Dose
    torch.cuda.synchronize()
    t = time.perf_counter()
    dose = Dose.from_geometry(ctx, spec, storage=storage)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t
    ms, runs, x, pl = timed_plans(ctx, dose, spec, st, args, args.warmup, args.steps)
    lam0, res = runs[-1]
    print(f"[bench] {spec.name} {storage}: {res.iterations} iterations, {ms:.2f} ms per plan", file=sys.stderr,
          flush=True)
    nt = args.trials_per_pass
    code = {"bf16": 1, "f16": 2}[storage]
    names = {"forward": f"fwd_wave_kernel<{nt}, 0, {16 if nt <= 2 else 8}, {code}, ",
             "adjoint": f"adj_kernel<{nt}, true, {code}, "}
    nv, nb, nnz = dose.nv, dose.nb, dose.nnz
    nr = nonempty_rows(dose)
    kern = kernel_table(runs, res, names, {"forward": forward_bytes16(nr, nb, nnz),
                                           "adjoint": adjoint_bytes16(nr, nb, nnz)})
    d16 = torch.empty(nv, dtype=torch.float32, device="cuda")
    d32 = torch.empty(nv, dtype=torch.float32, device="cuda")
    G16 = pl.objective(x, d16)
    G32_at = plan32.objective(x, d32)
    diff = (d16 - d32).abs().max().item()
    dmax = d32.abs().max().item()
    return {
        "storage": storage, "ms_per_plan": ms, "iterations": res.iterations, "status": res.status,
        "lambda0": lam0, "G_final": res.G_final, "solve_device_ms": res.device_ms, "dose_build_s": build_s,
        "kernels": kern,
        "vs_f32": {
            "time_ratio": ms / ms32,
            "dose_max_abs": diff, "dose_max_rel": diff / dmax if dmax > 0 else 0.0,
            "G_under_f32_D_rel": abs(G32_at - res32.G_final) / res32.G_final,
            "G_stored_vs_f32_rel": abs(G16 - res32.G_final) / res32.G_final,
            "note": "dose of this plan's x under D~ and under float32 D (max over voxels, relative to the "
                    "largest dose); G of that x under float32 D and this plan's own G, each against the "
                    "float32 plan's final G",
        },
    }


def batch_form(ctx, args):
    """The batched re-plan workload: `args.batch` uneven instances (seeds
    100, 101, ...), each planned alone in turn and then all together with
    imrt_solve_batch; aggregate rates of the batched solve."""
    import numpy as np
    import torch

    from paper_0908_4421_amd.imrt import Dose, Plan
    from workloads import PAPER_SCALE_SETTINGS as st
    from workloads import batch_instances, penalty_table, power_start_vector
    specs = batch_instances(100, args.batch)
    torch.cuda.synchronize()
    t = time.perf_counter()
    doses = [Dose.from_geometry(ctx, sp) for sp in specs]
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t
    plans = []
    for d, sp in zip(doses, specs):
        pl = Plan(ctx, d)
        pl.set_structures(None, 4)
        pl.set_penalties(penalty_table(sp))
        plans.append(pl)
    t = time.perf_counter()
    lams = [pl.lambda0(torch.as_tensor(power_start_vector(d.nb, sp.seed).astype(np.float32)).cuda(),
                       st.power_iters)[0] for pl, d, sp in zip(plans, doses, specs)]
    torch.cuda.synchronize()
    lam_s = time.perf_counter() - t
    kw = dict(eps=st.eps, alpha=st.alpha, delta=st.delta, max_iter=st.max_iter, max_backtracks=st.max_backtracks)
    xs = [torch.full((d.nb,), st.x0, dtype=torch.float32, device="cuda") for d in doses]
    solo_ms = [0.0] * len(plans)

    def solo():
        out = []
        for i, (pl, x, lam) in enumerate(zip(plans, xs, lams)):
            x.fill_(st.x0)
            t0 = time.perf_counter()
            out.append(pl.solve(x, lambda0=lam, **kw)[0])
            solo_ms[i] = (time.perf_counter() - t0) * 1e3
        return out

    # one by one with the default (single-plan) partitions
    solo()   # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    solo()
    torch.cuda.synchronize()
    solo_default_s = time.perf_counter() - t
    solo_default_ms = list(solo_ms)
    for x in xs:
        x.fill_(st.x0)
    # launch-shape search (leaves the chosen partition on every matrix; the
    # one-by-one solves below use it too)
    torch.cuda.synchronize()
    t = time.perf_counter()
    part = Plan.autotune_batch(plans, xs, eps=st.eps, alpha=st.alpha, lambda0s=lams, delta=st.delta,
                               tune_iters=args.tune_iters, max_iter=st.max_iter) if args.tune_iters >= 0 else None
    tune_s = time.perf_counter() - t

    def batched():
        for x in xs:
            x.fill_(st.x0)
        return [r for r, _ in Plan.solve_batch(plans, xs, lambda0s=lams, **kw)]

    solo()   # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    rs = solo()
    torch.cuda.synchronize()
    solo_s = time.perf_counter() - t
    x_solo = [x.clone() for x in xs]
    batched()   # warm-up
    times = []
    for _ in range(max(args.batch_steps, 1)):
        torch.cuda.synchronize()
        t = time.perf_counter()
        rb = batched()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
    batch_s = sorted(times)[len(times) // 2]
    same = all(a.iterations == b.iterations and a.G_final == b.G_final and torch.equal(xa, xb)
               for a, b, xa, xb in zip(rs, rb, x_solo, xs))
    nrs = [nonempty_rows(d) for d in doses]
    nbytes = sum(r.forward_passes * f32_forward(ctx, d.nb)[1](nr, d.nb, d.nnz) +
                 r.adjoint_passes * adjoint_bytes(nr, d.nb, d.nnz) for r, d, nr in zip(rb, doses, nrs))
    iters = sum(r.iterations for r in rb)
    print(f"[bench] batch of {len(specs)}: {iters} iterations, {batch_s * 1e3:.1f} ms batched, "
          f"{solo_default_s * 1e3:.1f} ms one by one", file=sys.stderr, flush=True)
    return {
        "workload": f"{len(specs)} uneven re-plans, seeds 100-{100 + len(specs) - 1}",
        "instances": len(specs),
        "nnz_total": sum(d.nnz for d in doses),
        "nnz_range": [min(d.nnz for d in doses), max(d.nnz for d in doses)],
        "matrix_MB_total": sum(16 * d.nnz for d in doses) / 1e6,
        "iterations_total": iters,
        "iterations_range": [min(r.iterations for r in rb), max(r.iterations for r in rb)],
        "batch_s": batch_s,
        "solo_sequential_s": solo_default_s,
        "solo_sequential_same_partition_s": solo_s,
        "speedup_vs_sequential": solo_default_s / batch_s,
        "plans_per_s": len(specs) / batch_s,
        "iters_per_s": iters / batch_s,
        "GB_s": nbytes / batch_s / 1e9,
        "frac_of_peak": nbytes / batch_s / 1e9 / HBM_PEAK_GBS,
        "bit_identical_to_solo": same,
        "dose_build_s": build_s,
        "lambda0_s": lam_s,
        "partition": {"adjoint_workgroups_per_plan": part[0] if part else None,
                      "forward_workgroups_per_plan": part[1] if part else None, "autotune_s": tune_s,
                      "autotune": "whole batch solved per candidate" if args.tune_iters == 0 else
                                  f"{args.tune_iters} iterations per candidate"},
        "per_plan": [{"nnz": d.nnz, "iterations": r.iterations, "solo_ms": a, "solo_same_partition_ms": b,
                      "adj_min_nnz": d.partition()[0], "fwd_blocks_per_wave": d.partition()[1]}
                     for d, r, a, b in zip(doses, rb, solo_default_ms, solo_ms)],
        "note": "times exclude the dose-matrix builds, the lambda_0 estimates and the launch-shape search "
                "(reported apart); "
                "GB/s counts the algorithmic bytes of every pass of every plan",
    }


def replan_form(ctx, plan, x, spec, st, args):
    """The paper's re-plan workload: the original plan's dose becomes every
    voxel's target (Eq. (1) with per-voxel T_j), re-optimised from x = x0 on
    the day's anatomy (target shrunk, bladder filled, rectum emptied)."""
    import numpy as np
    import torch

    from paper_0908_4421_amd.imrt import Dose, Plan
    from workloads import PTV, day_geometry, penalty_table, power_start_vector
    T = torch.empty(plan.dose.nv, dtype=torch.float32, device="cuda")
    plan.objective(x, T)
    T = T.cpu().numpy()
    day = day_geometry(spec)
    torch.cuda.synchronize()
    t = time.perf_counter()
    dose = Dose.from_geometry(ctx, day)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t
    p = Plan(ctx, dose)
    p.set_structures(None, 4)
    p.set_penalties(penalty_table(day))
    p.set_voxel_targets(T, T)
    v0 = torch.as_tensor(power_start_vector(dose.nb, day.seed).astype(np.float32)).cuda()
    xr = torch.empty(dose.nb, dtype=torch.float32, device="cuda")
    times = []
    for i in range(args.warmup + max(args.steps, 1)):
        xr.fill_(st.x0)
        torch.cuda.synchronize()
        t = time.perf_counter()
        lam, _ = p.lambda0(v0, st.power_iters)
        res, _ = p.solve(xr, eps=st.eps, alpha=st.alpha, lambda0=lam, delta=st.delta, max_iter=st.max_iter,
                         max_backtracks=st.max_backtracks)
        torch.cuda.synchronize()
        if i >= args.warmup:
            times.append(time.perf_counter() - t)
    ms = 1e3 * sum(times) / len(times)
    d = torch.empty(dose.nv, dtype=torch.float32, device="cuda")
    p.objective(xr, d)
    d = d.cpu().numpy()
    sid = dose.export(structures=True)["struct_id"]
    ptv = sid == PTV
    rel = np.abs(d[ptv] - T[ptv]) / np.maximum(T[ptv], 1e-30)
    # the warm-start variant of the line search (step 2 at alpha times the
    # previous accepted step), same stopping rule; one and two trial steps
    # per forward pass (the doubled first trial is often rejected, and with
    # two per pass its reduction needs no second pass)
    warm = {}
    for nt in (1, 2):
        wt = []
        for i in range(2):
            xr.fill_(st.x0)
            torch.cuda.synchronize()
            t = time.perf_counter()
            lam, _ = p.lambda0(v0, st.power_iters)
            rw, _ = p.solve(xr, eps=st.eps, alpha=st.alpha, lambda0=lam, delta=st.delta, max_iter=st.max_iter,
                            max_backtracks=st.max_backtracks, warm_start=True, trials_per_pass=nt)
            torch.cuda.synchronize()
            wt.append(1e3 * (time.perf_counter() - t))
        dw = torch.empty(dose.nv, dtype=torch.float32, device="cuda")
        p.objective(xr, dw)
        dw = dw.cpu().numpy()
        relw = np.abs(dw[ptv] - T[ptv]) / np.maximum(T[ptv], 1e-30)
        warm[f"trials_per_pass_{nt}"] = {"ms": wt[-1], "iterations": rw.iterations, "status": rw.status,
                                         "forward_passes": rw.forward_passes, "G_final": rw.G_final,
                                         "target_voxels_within_3pct": float(np.mean(relw <= 0.03))}
    nr = nonempty_rows(dose)
    nbytes = res.forward_passes * f32_forward(ctx, dose.nb)[1](nr, dose.nb, dose.nnz) + \
        res.adjoint_passes * adjoint_bytes(nr, dose.nb, dose.nnz)
    print(f"[bench] re-plan on {day.name}: {res.iterations} iterations, {ms:.2f} ms", file=sys.stderr, flush=True)
    return {
        "workload": f"{day.name}: targets = original plan's dose (per voxel), x0 = {st.x0}",
        "nb": dose.nb, "nnz": dose.nnz,
        "ms_per_replan": ms,
        "iterations": res.iterations,
        "status": res.status,
        "G_initial": res.G_initial,
        "G_final": res.G_final,
        "GB_s": nbytes / (ms / 1e3) / 1e9,
        "dose_build_s": build_s,
        "target_voxels_within_3pct": float(np.mean(rel <= 0.03)),
        "target_voxels_within_5pct": float(np.mean(rel <= 0.05)),
        "warm_start": warm,
        "note": "time per re-plan: lambda_0 estimate plus solve, matrix resident; the day's matrix build apart",
    }


SCENARIO3_NOTE = ("the paper's Table 1 scenario 3 has 6,453 beamlets, 143,329 voxels and 43.3 M nonzeros "
                  "(its own time is context only: other hardware, data and iteration count)")
COARSE_NOTE = ("the paper-scale phantom with unspecified tissue at twice the voxel size in each dimension "
               "(Section 3.1's reduction of the problem size): every 2x2x2 block of normal-tissue voxels is "
               "one voxel")


def shape_form(ctx, args, spec=None, note=SCENARIO3_NOTE):
    """A further float32 plan timed like the headline plan (by default the
    shape of the paper's largest scenario: about 300 nonzeros per voxel,
    0.6 GB of CSR and CSC, beyond the last-level cache); per-pass rates from
    HIP events."""
    import torch

    from paper_0908_4421_amd.imrt import Dose
    from workloads import PAPER_SCALE_SETTINGS as st
    from workloads import SCENARIO3_SHAPE
    spec = SCENARIO3_SHAPE if spec is None else spec
    torch.cuda.synchronize()
    t = time.perf_counter()
    dose = Dose.from_geometry(ctx, spec)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t
    ms, runs, x, pl = timed_plans(ctx, dose, spec, st, args, 1, max(1, min(args.steps, 3)))
    lam0, res = runs[-1]
    nv, nb, nnz = dose.nv, dose.nb, dose.nnz
    nr = nonempty_rows(dose)
    nt = args.trials_per_pass
    lay, fwd_model = f32_forward(ctx, nb)
    names = {"forward": f"fwd_wave_kernel<{nt}, 0, {16 if nt <= 2 else 8}, {lay}, ",
             "adjoint": f"adj_kernel<{nt}, true, 0, "}
    kern = kernel_table(runs, res, names, {"forward": fwd_model(nr, nb, nnz), "adjoint": adjoint_bytes(nr, nb, nnz)})
    print(f"[bench] {spec.name}: {res.iterations} iterations, {ms:.2f} ms per plan, forward "
          f"{kern['forward']['frac_of_peak']:.2f} / adjoint {kern['adjoint']['frac_of_peak']:.2f} of peak",
          file=sys.stderr, flush=True)
    return {
        "workload": spec.name,
        "nv": nv, "nb": nb, "nnz": nnz,
        "nonempty_rows": nr,
        "csr_csc_MB": (forward_bytes(nr, nb, nnz) + adjoint_bytes(nr, nb, nnz)) / 1e6,
        "ms_per_plan": ms,
        "iterations": res.iterations,
        "status": res.status,
        "iters_per_s": res.iterations / (ms / 1e3),
        "lambda0": lam0,
        "kernels": kern,
        "traffic": {k: traffic_from_profile(names[k], spec.name) for k in names},
        "dose_build_s": build_s,
        "note": note,
    }


def read_probe(ctx, gib=4, reps=5):
    """Achievable HBM read rate: the library's streaming-read probe over
    `gib` GiB (16 times the 256 MB last-level cache); the best of `reps`."""
    import torch

    from paper_0908_4421_amd.imrt import imrt_read_probe
    buf = torch.ones(gib * (1 << 30) // 4, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    gbs = imrt_read_probe(ctx.handle, buf.data_ptr(), buf.numel() * 4, reps)
    del buf
    torch.cuda.empty_cache()
    return gbs


def tile_order(nx, ny, nz, tx=4, ty=4, tz=2):
    """Grid voxel indices in tiles of tx x ty x tz voxels (x fastest inside a
    tile, tiles in x, y, z order): the row order of a built phantom."""
    import numpy as np
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    key = (((z // tz) * ((ny + ty - 1) // ty) + y // ty) * ((nx + tx - 1) // tx) + x // tx)
    inner = ((z % tz) * ty + y % ty) * tx + x % tx
    j = (x + nx * (y + ny * z)).ravel()
    return j[np.lexsort((inner.ravel(), key.ravel()))]


def shard_form(ctx, dose, spec, iters=100):
    """One GPU's share of a plan sharded by voxel rows over G GPUs (G = 2, 4,
    8): contiguous row ranges of the tile order holding equal numbers of
    nonzeros; the share with the most nonzeros, with its voxels' structures
    and penalties, solved as its own plan for a fixed number of iterations;
    the mean duration of its forward and adjoint passes (HIP events around
    every 7th launch), against the whole matrix solved the same way.  The
    all-reduces of G and g a sharded solve adds are not part of it."""
    import numpy as np
    import torch

    from paper_0908_4421_amd.imrt import Dose, Plan
    from workloads import penalty_table
    ex = dose.export(structures=True)
    nv, nb = dose.nv, dose.nb
    rp = ex["row_ptr"].astype(np.int64)
    lens = np.diff(rp)
    order = tile_order(spec.nx, spec.ny, spec.nz)
    table = penalty_table(spec)

    def measure(d, sid):
        p = Plan(ctx, d)
        p.set_structures(sid, len(table))
        p.set_penalties(table)
        x = torch.ones(d.nb, dtype=torch.float32, device="cuda")
        kw = dict(eps=1e-4, alpha=2.0, lambda0=2.0 ** -11, max_iter=iters, fixed_iters=True, profile=7)
        p.solve(x, **kw)
        x.fill_(1.0)
        res, _ = p.solve(x, **kw)
        tf, ta = 1e3 * res.forward_kernel_ms, 1e3 * res.adjoint_kernel_ms
        nr = nonempty_rows(d)
        bf = f32_forward(ctx, nb)[1](nr, nb, d.nnz)
        ba = adjoint_bytes(nr, nb, d.nnz)
        return {"rows": d.nv, "nnz": d.nnz, "forward_us": tf, "adjoint_us": ta,
                "forward_GB_s": bf / (tf * 1e-6) / 1e9, "adjoint_GB_s": ba / (ta * 1e-6) / 1e9}

    out = {"whole": measure(dose, None)}
    for G in (2, 4, 8):
        cum = np.concatenate([[0], np.cumsum(lens[order])])
        bounds = [0] + [int(np.searchsorted(cum, g * cum[-1] / G)) for g in range(1, G)] + [nv]
        nnz_g = [int(cum[bounds[g + 1]] - cum[bounds[g]]) for g in range(G)]
        g = int(np.argmax(nnz_g))
        rows = order[bounds[g]:bounds[g + 1]]
        sl = lens[rows]
        srp = np.zeros(len(rows) + 1, np.int64)
        np.cumsum(sl, out=srp[1:])
        idx = np.repeat(rp[rows] - srp[:-1], sl) + np.arange(srp[-1])
        d = Dose.from_csr(ctx, len(rows), nb, srp.astype(np.int32), ex["col_idx"][idx], ex["val"][idx])
        m = measure(d, ex["struct_id"][rows])
        m["share_of_nnz"] = m["nnz"] / dose.nnz
        out[f"{G}_gpus"] = m
        d.close()
        print(f"[bench] row share of {G} GPUs: {m['rows']} rows, {m['nnz']} nonzeros, forward "
              f"{m['forward_us']:.1f} us, adjoint {m['adjoint_us']:.1f} us", file=sys.stderr, flush=True)
    return out


def _pct(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v, dtype=np.float64), q)) if len(v) else None


def shared_live_time(live, patients):
    """Time during which live plans share a resident matrix.  live[i] =
    (start, end) of request i, patients[i] its patient.  Returns (sum over
    requests of the time another live plan of the same patient overlaps it,
    sum of live times, number of requests with such a partner)."""
    shared, total, partners = 0.0, 0.0, 0
    for i, (a, b) in enumerate(live):
        cuts = sorted((max(a, c), min(b, d)) for j, (c, d) in enumerate(live)
                      if j != i and patients[j] == patients[i] and c < b and d > a)
        covered, end = 0.0, a
        for c, d in cuts:
            if d > end:
                covered += d - max(c, end)
                end = d
        shared += covered
        total += b - a
        partners += bool(cuts)
    return shared, total, partners


def serve_stream(ctx, reqs, budget, paced, st, storage):
    """Submit `reqs` to a fresh server (at their arrival times when `paced`,
    all at once otherwise), wait for every plan; per-request times."""
    from paper_0908_4421_amd.imrt import Server
    srv = Server(ctx, budget_bytes=budget, max_live=64)
    kw = dict(storage=storage, x0=st.x0, eps=st.eps, alpha=st.alpha, delta=st.delta, max_iter=st.max_iter,
              max_backtracks=st.max_backtracks)
    t0 = time.perf_counter()
    tickets, sub = [], []
    last = t0
    for i, r in enumerate(reqs):
        if paced:
            dt = t0 + r.arrival_s - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
        sub.append((time.perf_counter() - t0) * 1e3)
        tickets.append(srv.submit(r.patient, r.spec, r.table, **kw))
        if time.perf_counter() - last > 30.0:   # long streams report as they go
            last = time.perf_counter()
            print(f"[bench] serve: {i + 1} of {len(reqs)} requests submitted after {last - t0:.0f} s",
                  file=sys.stderr, flush=True)
    got = [srv.wait(tk) for tk in tickets]
    span = time.perf_counter() - t0
    stats = srv.stats()
    srv.close()
    res = [g[0] for g in got]
    times = [g[1] for g in got]
    plan = [t.plan_ms for t in times]
    queue = [t.queue_ms for t in times]
    # how often live plans share a resident matrix: each request is live
    # from its admission to its result; a plan shares its matrix while
    # another live plan of the same patient overlaps it
    live = [(s0 + t.queue_ms, s0 + t.plan_ms) for s0, t in zip(sub, times)]
    shared_ms, live_ms, with_partner = shared_live_time(live, [r.patient for r in reqs])

    def pct(v):
        return {"n": len(v), "p50": _pct(v, 50), "p99": _pct(v, 99), "max": max(v) if v else None}
    # (the server does not report a plan's rows with nonzeros: its voxel
    # count stands in, which overstates the bytes of plans with empty rows)
    def fb(nv, nb, nnz):
        return f32_forward(ctx, nb)[1](nv, nb, nnz) if storage == "f32" else forward_bytes16(nv, nb, nnz)
    ab = adjoint_bytes if storage == "f32" else adjoint_bytes16
    nbytes = sum(x.forward_passes * fb(t.nv, t.nb, t.nnz) + x.adjoint_passes * ab(t.nv, t.nb, t.nnz)
                 for x, t in zip(res, times))
    its = sorted(x.iterations for x in res)
    status = {}
    for x in res:
        status[str(x.status)] = status.get(str(x.status), 0) + 1
    return {
        "requests": len(reqs),
        "replans": sum(r.replan for r in reqs),
        "span_s": span,
        "plans_per_s": len(reqs) / span,
        "time_to_plan_ms": pct(plan),
        "time_to_plan_converged_ms": pct([p for p, x in zip(plan, res) if x.status == 0]),
        "time_to_plan_capped_ms": pct([p for p, x in zip(plan, res) if x.status == 1]),
        "queue_ms": pct(queue),
        "time_to_plan_replans_ms": pct([p for p, r in zip(plan, reqs) if r.replan]),
        "shared_matrix": {"live_time_fraction": shared_ms / live_ms if live_ms > 0 else 0.0,
                          "requests_with_a_live_partner": with_partner},
        "iterations_total": sum(its),
        "iterations": {"p50": _pct(its, 50), "p99": _pct(its, 99), "max": its[-1]},
        "status_counts": status,
        "GB_s_voxel_count_bound": nbytes / span / 1e9,
        "peak_resident_GB": stats["peak_bytes"] / 1e9,
        "resident_matrices": stats["resident_matrices"],
    }


def serve_form(ctx, args):
    """The served re-plan workload: Poisson streams at each rate of
    `args.serve_rates` (requests / s) over `args.serve_seconds` seconds, 30 %
    of them re-plans of a resident patient with new thresholds, bfloat16
    dose matrices, admission against an HBM budget; then a burst of
    `args.serve_burst` requests submitted at once (the server's capacity)."""
    import torch

    from workloads import PAPER_SCALE_SETTINGS as st
    from workloads import served_requests
    free, _ = torch.cuda.mem_get_info()
    budget = int(min(288e9, 0.8 * free))
    out = {"storage": args.serve_storage, "budget_GB": budget / 1e9, "rates": {}}
    for rate in [float(r) for r in args.serve_rates.split(",") if r]:
        n = max(int(round(rate * args.serve_seconds)), 4)
        r = serve_stream(ctx, served_requests(rate, n, seed=int(rate * 10)), budget, True, st, args.serve_storage)
        out["rates"][f"{rate:g}"] = r
        print(f"[bench] serve {rate:g} req/s: {n} requests, p50 {r['time_to_plan_ms']['p50']:.1f} ms, "
              f"p99 {r['time_to_plan_ms']['p99']:.1f} ms to plan; converged p99 "
              f"{r['time_to_plan_converged_ms']['p99']} ms (n {r['time_to_plan_converged_ms']['n']}); "
              f"shared-matrix live fraction {r['shared_matrix']['live_time_fraction']:.3f}",
              file=sys.stderr, flush=True)
    if args.serve_burst > 0:
        r = serve_stream(ctx, served_requests(1.0, args.serve_burst, seed=99), budget, False, st,
                         args.serve_storage)
        out["burst"] = r
        print(f"[bench] serve burst of {args.serve_burst}: {r['plans_per_s']:.1f} plans/s", file=sys.stderr,
              flush=True)
    out["note"] = ("times from arrival (submission) to the plan on the host, including the dose-matrix build "
                   "of a new patient and the lambda_0 estimate; requests i use geometry seed 1000 + i; "
                   f"{args.serve_seconds:g} s of arrivals per rate")
    return out


def cpu_baseline_child(workload, repeats):
    """The FP64 oracle on the host: lambda_0 estimate plus a full solve of the
    workload to the stopping rule, on one core.

    Runs in a fresh interpreter that never touches the GPU (bench.py starts it
    before its own first GPU call), so the oracle's dose-matrix build may use
    a process pool; the timed part then runs pinned to one core with one
    BLAS/OpenMP thread.  Prints one JSON object."""
    import statistics

    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import model, phantom, solver
    from workloads import NAMED, PAPER_SCALE_SETTINGS, TINY_SETTINGS, penalty_table, power_start_vector, \
        start_point
    spec = NAMED[workload]
    st = TINY_SETTINGS if workload == "tiny" else PAPER_SCALE_SETTINGS
    t = time.perf_counter()
    D = phantom.build_dose_matrix(spec, workers=min(spec.n_beams, 16, os.cpu_count() or 1))
    build_s = time.perf_counter() - t
    pen = model.VoxelPenalties.from_structures(D.struct_id, penalty_table(spec))
    core = min(os.sched_getaffinity(0))
    os.sched_setaffinity(0, {core})
    runs = []
    with threadpool_limits(1):
        for _ in range(max(1, repeats)):
            t0 = time.perf_counter()
            lam_ref, _ = solver.lambda0_from_power_iteration(D.csr, pen, power_start_vector(D.nb, spec.seed),
                                                             st.power_iters)
            t1 = time.perf_counter()
            ref = solver.solve(D.csr, pen, start_point(D.nb, st), eps=st.eps, alpha=st.alpha, lambda0=lam_ref,
                               delta=st.delta, max_iter=st.max_iter, max_backtracks=st.max_backtracks,
                               fixed_iters=st.fixed_iters, keep_trace=False)
            t2 = time.perf_counter()
            runs.append((t2 - t0, t1 - t0, ref.iterations, ref.G))
    total = statistics.median(r[0] for r in runs)
    print(json.dumps({
        "value": total, "unit": "s", "cores": 1, "kind": "oracle",
        "sample": (f"{len(runs)} full plan(s) of {spec.name} (median): lambda_0 estimate ({st.power_iters} power "
                   f"iterations, {runs[-1][1]:.2f} s) plus the solve to the stopping rule, {runs[-1][2]} "
                   f"iterations; scipy.sparse float64, one thread pinned to one core; the oracle's matrix "
                   f"build ({build_s:.1f} s, process pool) not timed"),
        "oracle_iterations": runs[-1][2],
        "oracle_G_final": runs[-1][3],
        "lambda0": lam_ref,
        "runs_s": [r[0] for r in runs],
        "host_cpu": _cpu_model(),
        "host_nproc": os.cpu_count(),
    }), flush=True)


def cpu_baseline(workload, repeats):
    """Run cpu_baseline_child in a child interpreter and return its JSON."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-child", "--workload", workload,
           "--cpu-repeats", str(repeats)]
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    print(f"[bench] cpu baseline: the oracle on one host core ({workload})", file=sys.stderr, flush=True)
    out = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env, timeout=900)
    if out.returncode != 0:
        raise RuntimeError(f"cpu baseline failed ({out.returncode}):\n{out.stderr[-2000:]}")
    res = json.loads(out.stdout.strip().splitlines()[-1])
    print(f"[bench] cpu baseline: {res['value']:.2f} s per plan, {res['oracle_iterations']} iterations",
          file=sys.stderr, flush=True)
    return res


def kernel_source_hash():
    """sha256 of the kernel sources; recorded with every counter summary."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def summarize_pmc(folder):
    """Median per dispatch of every counter and kernel in the rocprofv3 CSV
    counter files under `folder` (dispatches that did no work are skipped: a
    value below 1 % of the kernel's largest)."""
    import csv
    import glob
    import statistics
    from collections import defaultdict
    per = defaultdict(float)
    for path in sorted(glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)):
        with open(path, newline="") as f:
            for row in csv.DictReader(f):
                key = (row["Dispatch_Id"], row["Kernel_Name"], row["Counter_Name"])
                per[key] += float(row["Counter_Value"])
    by = defaultdict(list)
    for (_, kern, ctr), v in per.items():
        by[(kern, ctr)].append(v)
    print(f"kernel_source_sha256 = {kernel_source_hash()}")
    for (kern, ctr), vals in sorted(by.items()):
        top = max(vals)
        work = [v for v in vals if v >= 0.01 * top] or vals
        print(f"counter | {kern} | {ctr} | dispatches {len(vals)} | working {len(work)} | "
              f"median {statistics.median(work):.1f} | mean {statistics.fmean(work):.1f}")


def traffic_from_profile(kernel_key, workload="prostate_160x104x80_2.5mm_9field"):
    """HBM bytes per launch of the named kernel on the named workload from the
    committed counter summary: FETCH_SIZE and WRITE_SIZE medians (KiB per
    dispatch), each scaled by the factor a plain device copy of known size
    gave for the same counter.  None when there is no summary for the
    workload or the kernel sources changed since."""
    try:
        with open(TRAFFIC_PROFILES[workload]) as f:
            lines = f.read().splitlines()
    except (KeyError, OSError):
        return None
    kv = {}
    ctr = {}
    for ln in lines:
        if ln.startswith("counter | "):
            parts = [p.strip() for p in ln.split("|")]
            if kernel_key in parts[1]:
                ctr[parts[2]] = float(parts[5].split()[1])
        elif " = " in ln and not ln.startswith("#"):
            k, v = ln.split(" = ", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_hash():
        return None
    if "FETCH_SIZE" not in ctr or "WRITE_SIZE" not in ctr:
        return None
    return (ctr["FETCH_SIZE"] * 1024 * float(kv["fetch_factor"]) +
            ctr["WRITE_SIZE"] * 1024 * float(kv["write_factor"]))


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="paper", choices=["paper", "tiny", "small", "scenario3"])
    ap.add_argument("--trials-per-pass", type=int, default=1)
    ap.add_argument("--cpu-repeats", type=int, default=1,
                    help="full oracle plans timed for the CPU baseline (median); one takes about 20 s")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--batch", type=int, default=32, metavar="N",
                    help="also time the batched re-plan workload of N uneven instances (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--tune-iters", type=int, default=0,
                    help="iterations per candidate of the batch's launch-shape search (0: the whole batch "
                         "solved per candidate; negative: no search, the default partition)")
    ap.add_argument("--no-shard", action="store_true",
                    help="skip the timing of one GPU's row share of the plan")
    ap.add_argument("--no-coarse", action="store_true",
                    help="skip the paper-scale plan with coarse unspecified tissue")
    ap.add_argument("--no-shape", action="store_true",
                    help="skip the plan on the shape of the paper's largest scenario")
    ap.add_argument("--no-replan", action="store_true",
                    help="skip the re-plan towards the original plan's dose on the day's anatomy")
    ap.add_argument("--serve-rates", default="2,5,10,20",
                    help="Poisson arrival rates (requests / s) of the served re-plan workload ('' : skip)")
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="seconds of arrivals per rate")
    ap.add_argument("--serve-burst", type=int, default=64, help="requests submitted at once after the streams")
    ap.add_argument("--serve-storage", default="bf16", choices=["f32", "bf16", "f16"])
    ap.add_argument("--forms", default="bf16,f16",
                    help="16-bit storage forms timed beside the float32 plan (comma list, or 'none')")
    ap.add_argument("--profile-every", type=int, default=31, metavar="N",
                    help="HIP events around every N-th forward and adjoint launch of the timed plans (31: "
                         "coprime with the 32-iteration batches the solver enqueues, so the samples fall at "
                         "every position of a batch)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (calibrates HBM byte counters)")
    ap.add_argument("--summarize-pmc", metavar="DIR",
                    help="only print per-kernel medians of the rocprofv3 CSV counter files under DIR")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc)
        return
    if args.cpu_baseline_child:
        cpu_baseline_child(args.workload, args.cpu_repeats)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs the solver on exactly one GPU and has no multi-GPU path; the row_shards object "
              "of its output times one GPU's share of a plan sharded by voxel rows.", file=sys.stderr)
        sys.exit(2)

    # the oracle runs first, in a child interpreter, before this process
    # touches the GPU
    cpu = None if (args.no_cpu_baseline or args.copy_calibration) else cpu_baseline(args.workload, args.cpu_repeats)

    import numpy as np
    import torch

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        reps = 5
        t = time.perf_counter()
        for _ in range(reps):
            dst.copy_(src)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / reps
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "reps": reps,
                          "GB_s_read_plus_write": 8 * n / dt / 1e9}), flush=True)
        return

    from paper_0908_4421_amd.imrt import Context, Dose
    from workloads import NAMED, PAPER_SCALE_SETTINGS, TINY_SETTINGS

    spec = NAMED[args.workload]
    st = TINY_SETTINGS if args.workload == "tiny" else PAPER_SCALE_SETTINGS
    ctx = Context(0)
    torch.cuda.synchronize()
    t = time.perf_counter()
    dose = Dose.from_geometry(ctx, spec)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t
    ms_per_step, runs, x, plan = timed_plans(ctx, dose, spec, st, args, args.warmup, args.steps)
    lam0, res = runs[-1]
    print(f"[bench] {spec.name}: {res.iterations} iterations, {ms_per_step:.2f} ms per plan", file=sys.stderr,
          flush=True)

    nv, nb, nnz = dose.nv, dose.nb, dose.nnz
    nr = nonempty_rows(dose)
    wave = ctx.get_option("fwd_wave")
    nt = args.trials_per_pass
    lay, fwd_model = f32_forward(ctx, nb)
    names = {"forward": f"fwd_wave_kernel<{nt}, 0, {16 if nt <= 2 else 8}, {lay}, " if wave else f"fwd_kernel<{nt}>(",
             "adjoint": f"adj_kernel<{nt}, true, 0, "}
    kern = kernel_table(runs, res, names, {"forward": fwd_model(nr, nb, nnz),
                                           "adjoint": adjoint_bytes(nr, nb, nnz)})
    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    probe = read_probe(ctx)
    roofline = {"bound": "hbm", "achieved": kern[dom]["GB_s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": kern[dom]["GB_s"] / HBM_PEAK_GBS, "traffic": traffic_from_profile(names[dom], spec.name),
                "kernel": kern[dom]["kernel"], "read_probe_GB_s": probe,
                "frac_of_read_probe": kern[dom]["GB_s"] / probe}

    out = {
        "metric": "time-to-plan (s) + SpMV HBM GB/s vs peak, 9-field 2.5mm; p99 served re-plan",
        "value": ms_per_step / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": spec.name, "nv": nv, "nonempty_rows": nr, "nb": nb, "nnz": nnz, "delta": st.delta,
                   "x0": st.x0, "eps": st.eps, "alpha": st.alpha, "lambda0": lam0,
                   "trials_per_pass": args.trials_per_pass,
                   "launch": {k: ctx.get_option(k) for k in ("fwd_wg_per_cu", "adj_wg_per_cu", "adj_min_nnz",
                                                             "fwd_col16", "batch_iters", "fwd_wave", "adj_xcd",
                                                             "stream_nt")}},
        "iterations": res.iterations,
        "iters_per_s": res.iterations / (ms_per_step / 1e3),
        "forward_passes": res.forward_passes,
        "adjoint_passes": res.adjoint_passes,
        "status": res.status,
        "G_final": res.G_final,
        "solve_device_ms": res.device_ms,
        "dose_build_s": build_s,
        "kernels": kern,
        "kernel_timing": f"HIP events around every {args.profile_every}-th launch of the timed plans",
        "roofline": roofline,
        "cpu_baseline": None,
    }
    if not args.no_replan:
        out["replan"] = replan_form(ctx, plan, x, spec, st, args)
    if not args.no_shard:
        out["row_shards"] = shard_form(ctx, dose, spec)
    if not args.no_shape and args.workload == "paper":
        out["scenario3_shape"] = shape_form(ctx, args)
    if not args.no_coarse and args.workload == "paper":
        from workloads import PAPER_SCALE_COARSE
        out["coarse_normal"] = shape_form(ctx, args, PAPER_SCALE_COARSE, COARSE_NOTE)
    forms = [f for f in args.forms.split(",") if f and f != "none"]
    if forms:
        out["forms"] = {f: storage_form(ctx, spec, st, args, f, plan, res, ms_per_step) for f in forms}
    if args.batch > 0:
        out["batch"] = batch_form(ctx, args)
    if args.serve_rates or args.serve_burst > 0:
        out["serve"] = serve_form(ctx, args)
    if cpu is not None:
        cpu["lambda0_matches"] = cpu["lambda0"] == lam0
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
