"""Benchmark: PDRQS1 iterations/s on one MI355X at 512^2 x 720 angles x 768 bins.

Workload (synthetic, seeded): a 512 x 512 FP32 random-ellipse phantom with two
metal discs (radius U[8, 20] px, density 20x the tissue maximum), 720 angles on
[0, pi), 768 bins; bins whose rays touch metal are inequality constraints
with lower bound 0.95 x the tissue-only projection, L2 fit elsewhere with 0.5 %
Gaussian noise; alpha = 0.005.  The sinogram, trace and bounds are built with
the library's own projector.

A step is one PDRQS1 iteration (R_h^* with the u_tmp epilogue, preconditioner
FFT pair, R_h, sinogram and gradient-side resolvents), run on inputs resident
in HBM.  Setup (normalization and c power iterations, 30 steps each) is timed
separately.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PD iterations/s and R+R* pairs/s (Gvox·angles/s) at 512²×720, % HBM roofline"
N_IMG, N_ANG, N_BIN = 512, 720, 768
# Published MI355X peaks used for the roofline fields.
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
# Plain VALU issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-instructions/s.
VALU_LANE_INSTR_PER_S = 256 * 4 * 16 * 2.4e9
# Algorithmic FP32 work of one pixel-angle pair in R_h or R_h^*: the step of
# the bin coordinate (1 add), the weight application (1 - alpha) v_k +
# alpha v_{k+1} as v_k + alpha (v_{k+1} - v_k) (subtract, multiply-add: 3)
# and the accumulation (1 add): 5 flops.
FLOPS_PER_PAIR = 5.0
# Algorithmic HBM bytes of one R_h launch inside the iteration: read the image
# once; read the target and vb1 and write vb1 and s1 once per bin (the fused
# sinogram-side update), plus the packed trace mask.
def radon_fwd_bytes(n, N, M):
    return 4.0 * (n * n + 4 * N * M) + N * ((M + 31) // 32) * 4.0


# ... of the gradient-side update when it runs inside R_h's launch: read vb2,
# write vb2 and s2 (two components each); the image is R_h's read.
def tv_fused_bytes(n):
    return 4.0 * 6 * n * n


# ... of one R_h^* launch inside the iteration: read s1 once, write the
# image (its angle slices' partial images are written and read once more by
# the preconditioner's row pass; counted there).
def radon_adj_bytes(n, N, M):
    return 4.0 * (N * M + n * n)


# ... of the preconditioner pair: u_tmp (formed from the slices as it is read)
# and the field s2 for its divergence, u, u_new, and the complex half
# spectrum written and read once by the column pass and once more by the
# inverse rows: 4 (n^2 (1 + 2 + 1 + 1) + 4 n (n/2 + 1)) bytes.
def fft_pair_bytes(n):
    return 4.0 * (5 * n * n + 4 * n * (n // 2 + 1))


PROFILES = os.path.join(ROOT, "profiles")


def profile_records(workload: str = "512x720x768"):
    """The committed counter records of a workload (n x N x M; each None
    when missing or taken on other kernel sources)."""
    from paper_1810_03275_amd.profiling import load_record
    stem = os.path.join(PROFILES, f"pdrqs1_{workload}_")
    return {"sq": load_record(stem + "sq_counters.json"),
            "tcc": load_record(stem + "tcc_counters.json"),
            "mix": load_record(stem + "valu_mix.json"),
            "traffic": load_record(stem + "traffic.json")}


def valu_busy_frac(mix, duration_s, rates):
    """The share of the chip's VALU capacity over a kernel's duration that
    its VALU instructions occupy, each type priced at the lane rate the
    probes measured: FP32 adds at the add probe's, FP32 multiplies and FMAs
    at the FMA probe's, 64-bit integer instructions at the 64-bit add
    probe's when that is slower than the 32-bit integer probe, and every other
    VALU instruction (integer, conversion, move, select, compare) at the
    32-bit integer probe's, which makes the figure an upper bound.  Also the
    FP32 share of the kernel's VALU instructions."""
    if not mix or not rates:
        return None, None
    add = mix["SQ_INSTS_VALU_ADD_F32"]
    fma = mix["SQ_INSTS_VALU_FMA_F32"] + mix["SQ_INSTS_VALU_MUL_F32"]
    i64 = mix["SQ_INSTS_VALU_INT64"]
    other = max(mix["SQ_INSTS_VALU"] - add - fma - i64, 0.0)
    slow = rates["xad_u32"]
    seconds = 64.0 * (add / rates["add_f32"] + fma / rates["fma_f32"]
                      + i64 / min(rates["add_u64"], slow) + other / slow)
    return round(seconds / duration_s, 4), round((add + fma) / mix["SQ_INSTS_VALU"], 4)


def kernel_roofline(recs, prefix, suffix, duration_s, flops, alg_bytes, bound, peak, unit,
                    rates=None):
    """The roofline object of one kernel: achieved = algorithmic work per
    launch / its average duration (HIP events), against the published peak;
    with the committed counters: the HBM bytes per launch, the VALU issue
    fraction (SQ_INSTS_VALU wave-instructions x 64 lanes against 256 CUs x 4
    SIMDs x 16 lanes x 2.4 GHz, i.e. 4 cycles per wave-instruction), the VALU
    busy fraction priced per instruction type at the measured probe rates
    (`rates`: lane-instructions/s per probe kind) and the L2 hit rate (TCC hits
    over hits + misses)."""
    from paper_1810_03275_amd.profiling import find_kernel
    if bound == "hbm":
        achieved = alg_bytes / duration_s / 1e9
    else:
        achieved = flops / duration_s / 1e12
    out = {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
           "frac": round(achieved / peak, 4), "duration_us": round(duration_s * 1e6, 2),
           "algorithmic_bytes": alg_bytes,
           "hbm_gbs_algorithmic": round(alg_bytes / duration_s / 1e9, 1)}
    tr = find_kernel(recs["traffic"], prefix, suffix)
    out["traffic"] = (tr["fetch_bytes"] + tr["write_bytes"]) if tr else None
    out["kernel"] = tr["name"] if tr else prefix + "..." + suffix
    if tr:
        out["hbm_gbs_counters"] = round(out["traffic"] / duration_s / 1e9, 1)
        out["hbm_frac_counters"] = round(out["traffic"] / duration_s / 1e9 / PEAK_HBM_GBS, 4)
    sq = find_kernel(recs["sq"], prefix, suffix)
    out["valu_issue_frac"] = (round(sq["SQ_INSTS_VALU"] * 64 / duration_s / VALU_LANE_INSTR_PER_S,
                                    4) if sq else None)
    out["valu_busy_frac"], out["valu_fp32_share"] = valu_busy_frac(
        find_kernel(recs["mix"], prefix, suffix), duration_s, rates)
    tc = find_kernel(recs["tcc"], prefix, suffix)
    if tc and (tc.get("TCC_HIT_sum", 0) + tc.get("TCC_MISS_sum", 0)) > 0:
        out["l2_hit_rate"] = round(tc["TCC_HIT_sum"] / (tc["TCC_HIT_sum"] + tc["TCC_MISS_sum"]), 4)
    else:
        out["l2_hit_rate"] = None
    return out


def fwd_kernel(lay, tun):
    """Name prefix and suffix of the R_h kernel a solver's iteration runs:
    the multi-angle walk with its angles per walk and the fused
    gradient-side update (or not), else the one-angle walk."""
    w = lay["angles_per_walk"]
    if w == 1:
        return "ctpd::k_radon_fwd<", ">"
    return f"ctpd::k_radon_fwd_multi<{w}", "true>" if tun["tv_blocks"] > 0 else "false>"


def adj_kernel(lay):
    """Name prefix and suffix of the R_h^* kernel a solver's iteration runs:
    mirror pairs (with their pixels per thread) or one angle at a time."""
    per = lay["bp_angles_per_position"]
    if per == 2:
        return "ctpd::k_radon_adj_pair<", f", {lay['bp_pair_pixels']}>"
    return "ctpd::k_radon_adj", "_adj"


def fft_pair_traffic(recs, lay):
    """Counter HBM bytes of the preconditioner's three kernels as the
    iteration runs them (the row pass that sums lay's slice count), or None."""
    from paper_1810_03275_amd.profiling import find_kernel
    S = lay["bp_slices"]
    parts = [find_kernel(recs["traffic"], "ctpd::k_fft_rows_fwd<", f", {S if S > 1 else 0}>"),
             find_kernel(recs["traffic"], "ctpd::k_fft_cols<"),
             find_kernel(recs["traffic"], "ctpd::k_fft_rows_inv<")]
    if any(p is None or p["fetch_bytes"] is None or p["write_bytes"] is None for p in parts):
        return None
    return sum(p["fetch_bytes"] + p["write_bytes"] for p in parts)


def _dpm_levels(path):
    """The levels of an amdgpu pp_dpm_* file, in MHz, and the current one."""
    levels, cur = [], None
    for line in open(path).read().splitlines():
        parts = line.split()
        if len(parts) >= 2 and parts[1].lower().endswith("mhz"):
            mhz = int(parts[1][:-3])
            levels.append(mhz)
            if "*" in parts[2:]:
                cur = mhz
    return levels, cur


def system_info(torch):
    """GPU SKU, ROCm/HIP version and the clock levels the amdgpu driver lists
    in sysfs (read as files: no tool process is started, so that the benchmark
    also runs unchanged under a profiler)."""
    import glob
    p = torch.cuda.get_device_properties(0)
    info = {"gpu": p.name, "arch": getattr(p, "gcnArchName", None),
            "compute_units": p.multi_processor_count,
            "memory_gib": round(p.total_memory / 2 ** 30, 1), "hip": torch.version.hip,
            "torch": torch.__version__}
    clocks = {}
    try:
        for dev in sorted(glob.glob("/sys/class/drm/card*/device")):
            for dom in ("sclk", "mclk"):
                f = os.path.join(dev, f"pp_dpm_{dom}")
                if os.path.exists(f) and dom not in clocks:
                    levels, cur = _dpm_levels(f)
                    clocks[dom] = {"levels_mhz": levels, "current_mhz": cur}
    except (OSError, ValueError) as e:   # the clocks are informational
        clocks["error"] = type(e).__name__
    info["clocks"] = clocks or "unavailable (no pp_dpm files)"
    return info


def build_inputs(ct, torch, w, plan=None):
    dev = torch.device("cuda")
    t = lambda a: torch.from_numpy(a.astype("float32")).to(dev)
    if plan is None:
        plan = ct.Plan(w.n, w.n_angles, w.n_bins)
    tissue_proj = plan.radon_fwd(t(w.tissue))
    clean = plan.radon_fwd(t(w.phantom))
    metal_proj = plan.radon_fwd(t(w.metal.astype("float32")))
    sigma_n = w.noise_level * float(tissue_proj.max())
    u0 = (clean + sigma_n * t(w.noise)).contiguous()
    mask = metal_proj > 0
    bound = torch.where(mask, 0.95 * tissue_proj, torch.zeros_like(tissue_proj)).contiguous()
    return plan, u0, ct.pack_mask(mask), bound, t(w.start_norm), t(w.start_precond)


def batched_run(ct, torch, iters: int, count: int = 64):
    """The uneven batch: 64 slices, n from {256, 384, 512, 768, 1024}, N = 1.4 n,
    M = 1.5 n, 0-3 metal discs; every batch (one per shape) advances with one
    launch per kernel and all batches replay as one HIP graph.  Times `iters`
    iterations after setup and 2 warm-up iterations."""
    import synth
    shapes = synth.batched_shapes(count)
    plans, groups = {}, {}
    for i, sh in enumerate(shapes):
        w = synth.batched_workload(i, sh)
        key = sh[:3]
        if key not in plans:
            plans[key] = ct.Plan(*key)
        plan, u0, mask, bound, _, _ = build_inputs(ct, torch, w, plans[key])
        groups.setdefault(key, []).append((u0, mask, bound, w.alpha))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solvers = []
    for key, items in groups.items():
        solvers.append(ct.SolverBatch(plans[key], [x[0] for x in items], items[0][3],
                                      [x[1] for x in items], [x[2] for x in items]))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    grp = ct.SolverGroup(solvers)
    grp.step(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    grp.step(iters)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    grp.close()
    pairs = sum(n * n * N for (n, N, M, _) in shapes)
    layout = {f"{k[0]}x{k[1]}x{k[2]}": dict(sv.layout(), problems=len(groups[k]))
              for k, sv in zip(groups, solvers)}
    return {"workload": f"{count} slices, n in {{256,384,512,768,1024}}, N=1.4n, M=1.5n, "
                        "0-3 metal discs, alpha=0.005",
            "iterations": iters, "ms_per_iteration": round(1e3 * dt / iters, 3),
            "it_per_s": round(iters / dt, 2),
            "gvox_angles_per_s": round(2 * pairs * iters / dt / 1e9, 1),
            "pairs_per_pass": pairs, "setup_s": round(setup_s, 3), "batches": layout}


def unrolled_run(ct, torch, K: int = 50, every: int = 10, count: int = 8):
    """Differentiation workload: 8 slices of 1024^2, 1440 angles x 1536 bins
    (random-ellipse phantoms, 1 % noise, alpha = 0.01) as one batch; K
    unrolled PDRQS1 iterations forward (checkpoints every `every`) and the
    reverse sweep for an MSE loss against the clean phantoms."""
    import synth
    ws = [synth.workload("C4", i) for i in range(count)]
    plan = ct.Plan(ws[0].n, ws[0].n_angles, ws[0].n_bins)
    sinos, truths = [], []
    for w in ws:
        _, u0, _, _, _, _ = build_inputs(ct, torch, w, plan)
        sinos.append(u0)
        truths.append(torch.from_numpy(w.phantom.astype("float32")).cuda())
    sinos = torch.stack(sinos).requires_grad_(True)
    truths = torch.stack(truths)
    lam = torch.tensor(ws[0].alpha, device="cuda", requires_grad=True)
    # warm-up (setup, graph capture) on a short unroll
    u = ct.unrolled_pd(plan, sinos, lam, K=2, every=1)
    ((u - truths) ** 2).mean().backward()
    sinos.grad = None
    lam.grad = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u = ct.unrolled_pd(plan, sinos, lam, K=K, every=every)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss = ((u - truths) ** 2).mean()
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    pairs = count * ws[0].n ** 2 * ws[0].n_angles
    return {"workload": f"{count} x {ws[0].n}^2, {ws[0].n_angles} x {ws[0].n_bins}, K={K}, "
                        f"checkpoint every {every}, MSE loss",
            "forward_ms": round(1e3 * (t1 - t0), 2), "backward_ms": round(1e3 * (t2 - t1), 2),
            "backward_over_forward": round((t2 - t1) / (t1 - t0), 3),
            "gvox_angles_per_s_forward": round(2 * pairs * K / (t1 - t0) / 1e9, 1),
            "dL_dlambda": float(lam.grad), "loss": float(loss.detach())}


def large_run(ct, torch, iters: int, tune_cache=None, rates=None):
    """The largest single slice: 2048^2, 2880 angles x 3072 bins, 4 metal discs,
    alpha = 0.005; PDRQS1 iterations/s after setup and 10 warm-up iterations,
    per-phase kernel durations (HIP events) and the rooflines of R_h, R_h^*
    and the FFT pair (with the counters of this workload's profile records)."""
    import synth
    w = synth.workload("C5")
    plan, u0, mask, bound, x0, x1 = build_inputs(ct, torch, w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    launch = ct.Launch(tune_cache=tune_cache) if tune_cache else None
    sv = ct.Solver(plan, u0, w.alpha, mask, bound, start_norm=x0, start_precond=x1,
                   launch=launch)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    sv.step(10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sv.step(iters)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ph = sv.step_timed(5)
    pairs = float(w.n * w.n * w.n_angles)
    lay, tun = sv.layout(), sv.tuning()
    recs = profile_records(f"{w.n}x{w.n_angles}x{w.n_bins}")
    fwd_prefix, fwd_suffix = fwd_kernel(lay, tun)
    t_fwd, t_adj, t_fft = (ph[k] * 1e-3 for k in ("radon_fwd", "radon_adj", "precond"))
    adj_prefix, adj_suffix = adj_kernel(lay)
    fft = {"duration_us": round(t_fft * 1e6, 2), "bound": "hbm", "peak": PEAK_HBM_GBS,
           "unit": "GB/s", "algorithmic_bytes": fft_pair_bytes(w.n),
           "achieved": round(fft_pair_bytes(w.n) / t_fft / 1e9, 1)}
    fft["frac"] = round(fft["achieved"] / PEAK_HBM_GBS, 4)
    tb = fft_pair_traffic(recs, lay)
    fft["traffic"] = tb
    if tb:
        fft["hbm_frac_counters"] = round(tb / t_fft / 1e9 / PEAK_HBM_GBS, 4)
    return {"workload": "2048x2048, 2880 angles, 3072 bins, 4 metal discs, alpha=0.005",
            "iterations": iters, "it_per_s": round(iters / dt, 2),
            "ms_per_iteration": round(1e3 * dt / iters, 3), "setup_s": round(setup_s, 3),
            "gvox_angles_per_s": round(2 * pairs * iters / dt / 1e9, 1),
            "phase_us": {k: round(v * 1e3, 1) for k, v in ph.items()},
            "layout": lay, "tuning": tun,
            "roofline_radon_fwd": kernel_roofline(
                recs, fwd_prefix, fwd_suffix, t_fwd, FLOPS_PER_PAIR * pairs,
                radon_fwd_bytes(w.n, w.n_angles, w.n_bins)
                + (tv_fused_bytes(w.n) if tun["tv_blocks"] > 0 else 0.0), "alu", PEAK_FP32_TFLOPS,
                "TFLOP/s", rates),
            "roofline_radon_adj": kernel_roofline(
                recs, adj_prefix, adj_suffix, t_adj, FLOPS_PER_PAIR * pairs,
                radon_adj_bytes(w.n, w.n_angles, w.n_bins), "alu", PEAK_FP32_TFLOPS, "TFLOP/s",
                rates),
            "roofline_fft_pair": fft,
            "solve_1000_iterations_s": round(1000 * dt / iters + setup_s, 2)}


def precond_comparison(ct, torch, n: int = 256, lam: float = 0.005, kmax: int = 8192):
    """The preconditioning comparison of the thesis' results (objective value
    relative to the smallest attained, per iteration): PDRQS1 with the
    inverse-norm, the impulse-response and the circulant preconditioner, its
    PDRQ3 splitting, PDRQS1 with
    Richardson's M = m id, Algorithm
    CP, PDRQS2 and ADMM with 1 and 2 inner PCG steps (mu = 1), on an
    unconstrained random-ellipse phantom (n^2, N = 1.4 n,
    M = 1.5 n, 1 % noise).  Reports the iterations and seconds each method needs
    to bring (P - P*)/P* below 1, 1e-1 and 1e-2, with P* the smallest
    objective any method reached (the thesis' measure; P* being an attained
    value, errors near the end of the fastest method's run are not
    meaningful, hence no smaller tolerances)."""
    import synth
    w = synth.workload("C1", n=n, n_angles=int(round(1.4 * n)), n_bins=int(1.5 * n),
                       iters=kmax)
    plan, u0, _, _, x0, x1 = build_inputs(ct, torch, w)
    probe = ct.Solver(plan, u0, lam, start_norm=x0, start_precond=x1)
    inf = probe.info()
    marks = sorted(set([int(round(2 ** (i / 2))) for i in range(0, 60)
                        if 2 ** (i / 2) <= kmax] + [kmax]))
    curves, rates = {}, {}
    methods = {"pdrqs1": {}, "pdrqs1_impulse": {"method": "pdrqs1", "precond": "impulse"},
               "pdrqs1_circulant": {"method": "pdrqs1", "precond": "circulant"},
               "pdrqs3": {}, "richardson": {}, "cp": {}, "pdrqs2": {},
               "admm_cg1": {"method": "admm", "cg_steps": 1},
               "admm_cg2": {"method": "admm", "cg_steps": 2}}
    for method, opts in methods.items():
        kw = opts or {"method": method}
        # the kernel preconditioners have their own constant c
        cc = None if kw.get("precond") in ("impulse", "circulant") else inf["c"]
        sv = ct.Solver(plan, u0, lam, beta=inf["beta"], c=cc, **kw)
        done, vals = 0, []
        sv.step(10)   # warm-up (graph capture), then restart from zero
        sv = ct.Solver(plan, u0, lam, beta=inf["beta"], c=cc, **kw)
        torch.cuda.synchronize()
        t_run = 0.0
        for m in marks:
            t0 = time.perf_counter()
            sv.step(m - done)
            torch.cuda.synchronize()
            t_run += time.perf_counter() - t0
            done = m
            o = ct.objective(plan, u0, lam, sv.export()[0])
            vals.append(float(o[0] + o[1]))
        curves[method] = vals
        rates[method] = t_run / kmax
    best = min(min(v) for v in curves.values())
    out = {"workload": f"{n}x{n}, {w.n_angles} angles, {w.n_bins} bins, random-ellipse phantom, "
                       f"no metal, 1% noise, lambda={lam}",
           "P_star": best, "iterations": marks, "ms_per_iteration": {}, "to_tolerance": {}}
    for method, vals in curves.items():
        relerr = [(v - best) / best for v in vals]
        out["ms_per_iteration"][method] = round(1e3 * rates[method], 4)
        reach = {}
        for tol in (1.0, 1e-1, 1e-2):
            k = next((m for m, e in zip(marks, relerr) if e <= tol), None)
            reach[f"{tol:g}"] = None if k is None else {
                "iterations": k, "seconds": round(k * rates[method], 4)}
        out["to_tolerance"][method] = reach
        out.setdefault("relative_error", {})[method] = [float(f"{e:.2e}") for e in relerr]
    return out


def precond_comparisons(ct, torch, kmax: int):
    """The comparison at the workload's weight, at lambda = 0.1 (the weight of
    the thesis' ADMM figure) and at lambda = 0.3 (that of its preconditioning
    figure)."""
    return {f"lambda={lam:g}": precond_comparison(ct, torch, lam=lam, kmax=kmax)
            for lam in (0.005, 0.1, 0.3)}


def mar_pipeline(ct, torch, w, plan, u0, true_mask, iters: int, reps: int = 20):
    """The metal-artifact workflow of the thesis' real-metal experiment on the
    benchmark workload: an unconstrained reconstruction (iters PDRQS1
    iterations, no constraint), the metal-trace estimate from it (pixels above
    half the metal density, dilated by 5 px, projected, kappa = 1e-3;
    C = 0.8 u0 on the estimate), then the constrained reconstruction with the
    estimated D0 and C.  Reports the estimate's time (events on the current
    stream, average of `reps` calls), its recall and precision against the
    true trace, and how far the constrained reconstruction moves from the
    unconstrained one and from the one with the true D0 and C."""
    import numpy as np

    def bits(m):
        a = m.detach().cpu().numpy().astype(np.uint32)
        return np.unpackbits(a.view(np.uint8), axis=1, bitorder="little")[:, :w.n_bins].astype(bool)

    lam = w.alpha
    free = ct.Solver(plan, u0, lam)
    free.step(iters)
    u_free = free.export()[0].clone()
    thr = 0.5 * w.metal_value
    args = (plan, u_free, thr, 5, 1e-3)
    ct.estimate_d0(*args, u0=u0, c0=0.8)   # warm-up
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        chi, proj, est, bound = ct.estimate_d0(*args, u0=u0, c0=0.8)
    ev1.record()
    torch.cuda.synchronize()
    t_est = ev0.elapsed_time(ev1) / reps
    e, t = bits(est), bits(true_mask)
    hit = int(np.sum(e & t))
    con = ct.Solver(plan, u0, lam, est, bound)
    con.step(iters)
    u_con = con.export()[0]
    true_bound = torch.where(torch.from_numpy(t).cuda(), 0.8 * u0, torch.zeros_like(u0))
    ref = ct.Solver(plan, u0, lam, true_mask, true_bound.contiguous())
    ref.step(iters)
    u_ref = ref.export()[0]
    nrm = lambda x: float(torch.linalg.vector_norm(x))
    return {"workload": "512x512, 720 angles, 768 bins, 2 metal discs (density 20x tissue)",
            "threshold": thr, "dilation_px": 5, "kappa": 1e-3, "c0": 0.8,
            "iterations_per_solve": iters,
            "estimate_us": round(1e3 * t_est, 2),
            "marked_pixels": int(chi.sum().item()),
            "d0_bins": int(e.sum()), "true_trace_bins": int(t.sum()),
            "recall": round(hit / max(int(t.sum()), 1), 4),
            "precision": round(hit / max(int(e.sum()), 1), 4),
            "rel_change_vs_unconstrained": round(nrm(u_con - u_free) / nrm(u_free), 4),
            "rel_diff_vs_true_d0": round(nrm(u_con - u_ref) / nrm(u_ref), 4)}


def cpu_baseline(w, budget_s: float):
    """The FP64 oracle timed on this host on a bounded sample of the same
    workload (setup with beta and c given, not timed): PDRQS1 iterations for
    about budget_s / 2 seconds on one core, then for as long with its
    projector pair split over angle blocks on all the host's cores (at most
    16, a GPU's share of the host) and numpy.fft on one thread."""
    import numpy as np
    from oracle import geometry, pdrq, radon
    from oracle.parallel import AngleBlocks
    g = geometry.Geometry(w.n, w.n_angles, w.n_bins)
    tissue = radon.radon_fwd(g, w.tissue)
    u0 = radon.radon_fwd(g, w.phantom) + w.noise_level * tissue.max() * w.noise
    mask = radon.radon_fwd(g, w.metal.astype(float)) > 0
    bound = np.where(mask, 0.95 * tissue, 0.0)
    prob = pdrq.Problem(g, u0, mask, bound, w.alpha)

    def rate(s, budget):
        st = pdrq.zero_state(s)
        t0 = time.perf_counter()
        k = 0
        while True:
            st = pdrq.step(s, st)
            k += 1
            if time.perf_counter() - t0 >= budget:
                break
        return k, time.perf_counter() - t0

    k1, dt1 = rate(pdrq.setup(prob, pdrq.Params(), beta=1.0e3, c=1.0), budget_s / 2)
    workers = max(1, min(16, os.cpu_count() or 1))
    ab = AngleBlocks(g, workers)
    try:
        ab.fwd(np.zeros((g.n, g.n)))   # start the worker processes
        kn, dtn = rate(pdrq.setup(prob, pdrq.Params(), beta=1.0e3, c=1.0, fwd=ab.fwd,
                                  adj=ab.adj), budget_s / 2)
    finally:
        ab.close()
    return {"value": kn / dtn, "unit": "it/s", "cores": workers, "kind": "oracle",
            "single_core_value": k1 / dt1, "host_cpus": os.cpu_count(),
            "sample": f"PDRQS1 iterations of the 512^2 x 720 x 768 workload in FP64 NumPy: "
                      f"{kn} in {dtn:.1f} s with the projector pair on {workers} worker "
                      f"processes, {k1} in {dt1:.1f} s on one core (setup with beta and c "
                      f"given, not timed)"}


def device_calibration(ct, torch):
    """The achievable FP32 VALU issue rate and HBM copy bandwidth, measured
    with the library's probes (HIP events, median of 5 launches)."""
    def timed(launch, reps=5):
        launch()
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            launch()
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        return sorted(ms)[reps // 2] * 1e-3

    blocks, iters = 8192, 4096
    out = torch.zeros(blocks, device="cuda")
    valu = {}
    for kind in ct.VALU_PROBE_KINDS:
        count = ct.valu_probe(blocks, 1, out, kind)  # count per round x iters below
        t = timed(lambda: ct.valu_probe(blocks, iters, out, kind))
        rate = count * iters * 64.0 / t
        valu[kind] = {"lane_instr_per_s": float(f"{rate:.4g}"),
                      "cycles_per_wave_instr": round(256 * 4 * 2.4e9 / (rate / 64.0), 3)}
    nbytes = 2 << 30  # 2 GiB each way: well beyond the 256 MB last-level cache
    src = torch.ones(nbytes // 4, device="cuda")
    dst = torch.empty_like(src)
    tc = timed(lambda: ct.copy_probe(src, dst, 8192))
    del src, dst
    gbs = 2 * nbytes / tc / 1e9
    return {"valu": valu, "copy_gbs": round(gbs, 1),
            "copy_frac_of_peak": round(gbs / PEAK_HBM_GBS, 4),
            "probes": "16 independent chains per lane of each instruction kind, 8192 x 256 "
                      "threads x 4096 rounds (cycles per wave-instruction per SIMD at 2.4 GHz); "
                      "a 2 GiB device copy with 16-byte accesses (read + write bytes)"}


def copy_calibration(torch):
    """A plain 64 MiB device copy, three times: the reference dispatch of
    known size that scales the FETCH_SIZE / WRITE_SIZE counters."""
    x = torch.ones(16 * 1024 * 1024, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--batched-iters", type=int, default=20,
                    help="timed iterations of the 64-slice uneven batch (0: skip)")
    ap.add_argument("--unrolled-iters", type=int, default=50,
                    help="unrolled iterations of the differentiation workload (0: skip)")
    ap.add_argument("--large-iters", type=int, default=50,
                    help="timed iterations at 2048^2 x 2880 x 3072 (0: skip)")
    ap.add_argument("--comparison-iters", type=int, default=8192,
                    help="iterations of the preconditioning comparison (0: skip)")
    ap.add_argument("--mar-iters", type=int, default=500,
                    help="iterations per solve of the metal-artifact workflow (0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 64 MiB device copy (for counter scaling)")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file of launch-choice tuning results to reuse (and extend)")
    ap.add_argument("--large-only", action="store_true",
                    help="run only the 2048^2 workload (--large-iters iterations) and print "
                         "its results (for profiling its kernels apart from the others)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU (asked for --gpus {args.gpus}); the "
              "library has no multi-GPU path (sharding by angles is a design, not code).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1810_03275_amd as ct
    import synth

    if args.large_only:
        out = {"large": large_run(ct, torch, max(args.large_iters, 1), args.tune_cache),
               "system": system_info(torch)}
        if args.copy_calibration:
            copy_calibration(torch)
        print(json.dumps(out), flush=True)
        return

    w = synth.workload("C2")
    plan, u0, mask, bound, x0, x1 = build_inputs(ct, torch, w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    launch = ct.Launch(tune_cache=args.tune_cache) if args.tune_cache else None
    sv = ct.Solver(plan, u0, w.alpha, mask, bound, start_norm=x0, start_precond=x1,
                   launch=launch)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    info = sv.info()

    # the iterations timed with HIP events on the solver's stream (the current
    # stream): median over repeats of blocks of iterations.  They run before
    # the warm-up and the timed steps: right after set-up the GPU's time per
    # iteration still falls for some 10-20 ms of sustained work (0.121 ->
    # 0.112 ms over the first 80 iterations, in the kernels themselves, not
    # between launches), which a short timed region would otherwise measure.
    reps, block = 25, 20
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record()
    for r in range(reps):
        sv.step(block)
        ev[r + 1].record()
    torch.cuda.synchronize()
    per = sorted(ev[r].elapsed_time(ev[r + 1]) / block for r in range(reps))
    event_ms = per[reps // 2]

    sv.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sv.step(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    it_s = args.steps / dt
    rec = sv.gap()

    # the FP64 record inside the loop: a record every 10 iterations
    t0 = time.perf_counter()
    for _ in range(10):
        sv.step(10)
        sv.gap()
    torch.cuda.synchronize()
    with_gap = 100 / (time.perf_counter() - t0)

    # per-phase kernel durations of the same iterations with the same
    # launches, HIP events on the solver's stream (the current stream)
    ph = sv.step_timed(args.kernel_reps)
    t_fwd = ph["radon_fwd"] * 1e-3
    t_adj = ph["radon_adj"] * 1e-3
    t_fft = ph["precond"] * 1e-3
    pairs = float(N_IMG * N_IMG * N_ANG)
    lay, tun = sv.layout(), sv.tuning()
    recs = profile_records()
    cal = device_calibration(ct, torch)
    rates = {k: v["lane_instr_per_s"] for k, v in cal["valu"].items()}
    fwd_prefix, fwd_suffix = fwd_kernel(lay, tun)
    roof = kernel_roofline(recs, fwd_prefix, fwd_suffix, t_fwd,
                           FLOPS_PER_PAIR * pairs, radon_fwd_bytes(N_IMG, N_ANG, N_BIN)
                           + (tv_fused_bytes(N_IMG) if tun["tv_blocks"] > 0 else 0.0), "alu",
                           PEAK_FP32_TFLOPS, "TFLOP/s", rates)
    adj_prefix, adj_suffix = adj_kernel(lay)
    roof_adj = kernel_roofline(recs, adj_prefix, adj_suffix, t_adj, FLOPS_PER_PAIR * pairs,
                               radon_adj_bytes(N_IMG, N_ANG, N_BIN), "alu", PEAK_FP32_TFLOPS,
                               "TFLOP/s", rates)
    fft = {"duration_us": round(t_fft * 1e6, 2), "bound": "hbm", "peak": PEAK_HBM_GBS,
           "unit": "GB/s", "algorithmic_bytes": fft_pair_bytes(N_IMG),
           "achieved": round(fft_pair_bytes(N_IMG) / t_fft / 1e9, 1)}
    fft["frac"] = round(fft["achieved"] / PEAK_HBM_GBS, 4)
    fft["traffic"] = fft_pair_traffic(recs, lay)
    fft["traffic_note"] = "sum of the median counter bytes of the in-path FFT kernels"
    if fft["traffic"]:
        fft["hbm_frac_counters"] = round(fft["traffic"] / t_fft / 1e9 / PEAK_HBM_GBS, 4)
    out = {
        "metric": METRIC,
        "value": round(it_s, 2),
        "unit": "it/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "512x512 random-ellipse phantom + 2 metal discs, 720 angles, "
                               "768 bins, alpha=0.005, inequality constraints on the metal trace",
                   "image": N_IMG, "angles": N_ANG, "bins": N_BIN, "alpha": w.alpha,
                   "iterations_per_solve": w.iters},
        "untimed_iterations_before_warmup": reps * block,
        "event_timing": {"repeats": reps, "iterations_per_repeat": block,
                         "median_ms_per_iteration": round(event_ms, 5),
                         "it_per_s": round(1e3 / event_ms, 1)},
        "it_per_s_with_record_every_10": round(with_gap, 1),
        "radon_pairs_per_s": round(2 * pairs / (t_fwd + t_adj) / 1e9, 2),
        "radon_pairs_unit": "Gvox*angles/s (R+R*)",
        "phase_us": {k: round(v * 1e3, 2) for k, v in ph.items()},
        "setup_ms": round(setup_s * 1e3, 2),
        "layout": lay, "tuning": tun,
        "beta": info["beta"], "c": info["c"],
        "gap_record": [float(x) for x in rec],
        "roofline": roof,
        "roofline_radon_adj": roof_adj,
        "roofline_fft_pair": fft,
        "system": system_info(torch),
        "device_calibration": cal,
    }
    if args.batched_iters > 0:
        del sv
        torch.cuda.empty_cache()
        out["batched"] = batched_run(ct, torch, args.batched_iters)
    if args.mar_iters > 0:
        out["mar_pipeline"] = mar_pipeline(ct, torch, w, plan, u0, mask, args.mar_iters)
    if args.comparison_iters > 0:
        torch.cuda.empty_cache()
        out["preconditioning"] = precond_comparisons(ct, torch, args.comparison_iters)
    if args.large_iters > 0:
        torch.cuda.empty_cache()
        out["large"] = large_run(ct, torch, args.large_iters, args.tune_cache, rates)
    if args.unrolled_iters > 0:
        torch.cuda.empty_cache()
        out["unrolled"] = unrolled_run(ct, torch, args.unrolled_iters)
    if args.copy_calibration:
        copy_calibration(torch)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
