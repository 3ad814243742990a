"""Throughput of the STAP hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large]

One step is one pass of the whole hot path (Doppler filtering, covariance
with loading, Cholesky weight solve with FP64 refinement, inner products and
power) over one synthetic datacube already resident in HBM, through
``stap_run``.  The metric is range-cell x DOF per second (R * D / step time)
for the mixed-precision path; the plain FP32 path is timed on the same cube
for the ratio.  Accuracy against the FP64 oracle is checked on sampled
training blocks (weights error and SINR loss), per-kernel durations come from
HIP events on the launch stream, and the CPU oracle is timed on a bounded
sample of the same workload.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

HBM_PEAK = 8.0e12        # B/s
FP32_PEAK = 157.3e12     # flop/s, MI355X published FP32 (vector and matrix)
BF16_PEAK = 2.5e15       # flop/s dense
FP64_PEAK = 78.6e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="large", choices=["small", "medium", "large", "xlarge", "uneven"])
    ap.add_argument("--precision", default=None, choices=["fp32", "bf16", "fp8"],
                    help="mixed-path precision (default: fp8 for xlarge, bf16 otherwise)")
    ap.add_argument("--refine", type=int, default=1)
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP32 leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-seconds-single", type=float, default=8.0,
                    help="seconds of the single-threaded oracle sample")
    ap.add_argument("--no-paper", action="store_true",
                    help="skip the leg on the paper's own cube (100 pulses x 1000 channels x 30000 samples)")
    ap.add_argument("--no-cfar", action="store_true", help="skip the CA-CFAR leg")
    return ap.parse_args()


WL = {"small": synth.SMALL, "medium": synth.MEDIUM, "large": synth.LARGE, "xlarge": synth.XLARGE}


def kernel_work(wl, precision, refine):
    """Algorithmic HBM bytes and flops (by arithmetic type) per launch of each
    kernel on one cube.  Flop counts are those of the method (one complex
    product per lower-triangle covariance element, 4/3 D^3 for the Cholesky,
    8 D^2 per right-hand side for a forward plus back solve), not of the
    implementation (which computes six BF16 products per element on the mixed
    path and whole diagonal tiles)."""
    C, P, R, T, B, S = wl.n_chan, wl.n_pulse, wl.n_range, wl.tdof, wl.n_block, wl.n_steer
    D, N = wl.dof, wl.n_cell
    sysn = P * B
    cube_b = C * P * R * 8
    snap_b = P * D * R * 8
    cov_b = sysn * D * D * 8
    cov_lower_b = sysn * D * (D + 1) // 2 * 8
    w_b = sysn * S * D * 8
    pw_b = P * S * R * 4
    herm = 8.0 * (D * (D + 1) / 2) * N * sysn
    chol = (4.0 / 3.0) * D ** 3 * sysn
    solves = 8.0 * D * D * S * sysn
    cov_key = {"fp32": "fp32", "bf16": "bf16", "fp8": "fp8"}[precision]
    # the inner products run on BF16 matrix cores on the mixed paths
    inner_key = "fp32" if precision == "fp32" else "bf16"
    return {
        "doppler": dict(bytes=cube_b + snap_b, fp32=5.0 * T * C * R * P * np.log2(P)),
        "covariance": {"bytes": snap_b + cov_b, cov_key: herm},
        "solve": dict(bytes=cov_lower_b + w_b, fp32=chol + solves * (1 + refine), fp64=solves * refine),
        # fused: snapshots in, weights out; covariance products plus the solve
        "covariance_solve": {"bytes": snap_b + w_b, cov_key: herm,
                             "fp32": chol + solves * (1 + refine), "fp64": solves * refine},
        "inner": {"bytes": snap_b + w_b + pw_b, inner_key: 8.0 * S * D * N * sysn},
    }


def cfar_work(wl, n_ref):
    """CA-CFAR on the power map: power in (4 B) and mask out (1 B) per cell,
    2 n_ref FP64 additions per cell."""
    cells = wl.n_pulse * wl.n_steer * wl.n_range
    return {"bytes": 5 * cells, "fp64_add": 2.0 * n_ref * cells}


# fp64_add: plain FP64 additions, one per lane per instruction, so half the
# FMA-counted FP64 peak
PEAKS = {"fp32": FP32_PEAK, "bf16": BF16_PEAK, "fp8": 5.0e15, "fp64": FP64_PEAK, "fp64_add": FP64_PEAK / 2}


def roofline_of(name, work, sec):
    """Bound of one kernel: max(bytes / HBM peak, sum over arithmetic types of
    flops / that type's peak).  frac = bound time / measured time; for a
    compute bound, achieved = all flops / time and peak = all flops / compute
    bound time (the blended peak of the kernel's own flop mix)."""
    t_hbm = work["bytes"] / HBM_PEAK
    flops = sum(v for k, v in work.items() if k in PEAKS)
    t_cmp = sum(v / PEAKS[k] for k, v in work.items() if k in PEAKS)
    if t_hbm >= t_cmp:
        ach = work["bytes"] / sec
        return dict(bound="hbm", achieved=ach / 1e9, peak=HBM_PEAK / 1e9, unit="GB/s", frac=ach / HBM_PEAK)
    ach = flops / sec
    peak = flops / t_cmp
    bound = "mfma" if name in ("covariance", "inner") else "alu"
    if name == "cfar":
        bound = "alu"
    return dict(bound=bound, achieved=ach / 1e12, peak=peak / 1e12, unit="TFLOP/s", frac=ach / peak)


PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_2203_06233_amd", "csrc")


def kernel_source_hash():
    """SHA-256 over the HIP sources of the library, in name order."""
    import hashlib
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hip", ".h")):
            h.update(f.encode())
            h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()


def measured_traffic(kernel, workload, precision, refine):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary for this workload (FETCH_SIZE + WRITE_SIZE, each scaled by what
    the counter reads for a copy of known size), or None when there is none
    or the kernel sources changed since the counters were taken."""
    path = os.path.join(PROFILES, f"{kernel}_{workload}_{precision}_r{refine}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith((" ", "#", "`")):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    try:
        if kv.get("source_sha256") != kernel_source_hash():
            return None
        return float(kv["traffic_bytes"])
    except (KeyError, ValueError):
        return None

def main():
    args = parse()
    if args.precision is None:
        args.precision = "fp8" if args.workload == "xlarge" else "bf16"
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); the path would shard "
              "by training blocks along range with no collective, which one GPU's share already shows",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2203_06233_amd import stap

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.workload == "uneven":
        wls = synth.uneven_batch(64)
    else:
        wls = [WL[args.workload]]
    t0 = time.perf_counter()
    cubes_np = [synth.make_cube(w) for w in wls]
    steers_np = [synth.steering(w) for w in wls]
    gen_s = time.perf_counter() - t0
    cubes = [torch.from_numpy(c).to(dev) for c in cubes_np]
    steers = [torch.from_numpy(v).to(dev) for v in steers_np]
    cells_dof = sum(w.cells_dof for w in wls)

    def mkprob(w, prec, refine):
        return stap.problem(w.n_chan, w.n_pulse, w.n_range, w.tdof, w.n_block, w.n_steer,
                            load_eps=w.load_eps, precision=prec, refine_steps=refine)

    def time_run(prec, refine):
        probs = [mkprob(w, prec, refine) for w in wls]
        runner = stap.Runner(probs, device=dev)
        powers = [torch.empty((w.n_pulse, w.n_steer, w.n_range), dtype=torch.float32, device=dev) for w in wls]
        weights = [torch.empty((w.n_pulse, w.n_block, w.n_steer, w.dof), dtype=torch.complex64, device=dev)
                   for w in wls]
        info = [torch.empty((w.n_pulse, w.n_block), dtype=torch.int32, device=dev) for w in wls]
        for _ in range(args.warmup):
            runner.run(cubes, steers, powers=powers, weights=weights, info=info)
        torch.cuda.synchronize()
        st = torch.cuda.current_stream()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t = time.perf_counter()
        ev0.record(st)
        for _ in range(args.steps):
            runner.run(cubes, steers, powers=powers, weights=weights, info=info)
        ev1.record(st)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t) / args.steps
        ev_ms = ev0.elapsed_time(ev1) / args.steps
        return wall, ev_ms, powers, weights, info

    wall_m, ev_m, powers, weights, info = time_run(args.precision, args.refine)
    # keep on the host only what the accuracy check reads: three sampled
    # training blocks of the first cube
    w0 = wls[0]
    N0 = w0.n_cell
    acc_blocks = sorted({0, w0.n_block // 2, w0.n_block - 1})
    out_w = {b: weights[0][:, b].cpu().numpy() for b in acc_blocks}
    out_power = {b: powers[0][:, :, b * N0:(b + 1) * N0].cpu().numpy() for b in acc_blocks}
    info_nonzero = int(sum(int((i != 0).sum().item()) for i in info))
    del powers, weights, info
    torch.cuda.empty_cache()

    plain = None
    if not args.no_plain:
        wall_p, ev_p, pw, ww, ii = time_run("fp32", 0)
        plain = dict(ms_per_step=wall_p * 1e3, value=cells_dof / wall_p)
        del pw, ww, ii
        torch.cuda.empty_cache()
    # the same precision without the refinement step, for context
    unrefined = None
    if not args.no_plain and args.refine > 0:
        wall_u, ev_u, pw, ww, ii = time_run(args.precision, 0)
        unrefined = dict(ms_per_step=wall_u * 1e3, value=cells_dof / wall_u)
        del pw, ww, ii
        torch.cuda.empty_cache()

    # per-kernel durations with HIP events on the launch stream (single cube)
    kern = {}
    roof = None
    if len(wls) == 1:
        w = wls[0]
        prob = mkprob(w, args.precision, args.refine)
        st = torch.cuda.current_stream()
        # the kernels stap_run launches: Doppler, fused covariance->solve (or,
        # for D > 128 and FP8, covariance then solve), inner products
        snap = stap.doppler(prob, cubes[0])
        calls = {"doppler": lambda: stap.doppler(prob, cubes[0], snap)}
        try:
            wts, inf = stap.covariance_solve(prob, snap, steers[0])
            calls["covariance_solve"] = lambda: stap.covariance_solve(prob, snap, steers[0], wts, inf)
            cov = None
        except stap.StapError as e:
            if e.code != -6:
                raise
            cov, dlt = stap.covariance(prob, snap)
            wts, inf = stap.solve_weights(prob, cov, steers[0])
            calls["covariance"] = lambda: stap.covariance(prob, snap, cov, dlt)
            calls["solve"] = lambda: stap.solve_weights(prob, cov, steers[0], wts, inf)
        pwr = stap.inner_products(prob, wts, snap)
        calls["inner"] = lambda: stap.inner_products(prob, wts, snap, pwr)
        work = kernel_work(w, args.precision, args.refine)
        if not args.no_cfar:
            # CA-CFAR on the power map (16 reference and 2 guard cells per
            # side, Pfa 1e-4 on exponential noise): the step after the chain
            from oracle import cfar as ocfar  # the closed-form threshold factor only
            alpha = ocfar.alpha_for_pfa(32, 1e-4)
            det = stap.cfar(prob, pwr, 16, 2, alpha)
            calls["cfar"] = lambda: stap.cfar(prob, pwr, 16, 2, alpha, det)
            work["cfar"] = cfar_work(w, 16)
        ksteps = max(1, min(args.steps, 20))
        for name, fn in calls.items():
            for _ in range(2):
                fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(ksteps):
                fn()
            e1.record(st)
            torch.cuda.synchronize()
            sec = e0.elapsed_time(e1) / ksteps / 1e3
            kern[name] = dict(ms=sec * 1e3, **roofline_of(name, work[name], sec))
        dom = max((k for k in kern if k != "cfar"), key=lambda k: kern[k]["ms"])
        r = kern[dom]
        roof = dict(kernel=dom, bound=r["bound"], achieved=r["achieved"], peak=r["peak"], unit=r["unit"],
                    frac=r["frac"], traffic=measured_traffic(dom, w.name, args.precision, args.refine))
        del snap, wts, inf, pwr, cov
        calls.clear()
        torch.cuda.empty_cache()

    # accuracy against the FP64 oracle on sampled training blocks
    from oracle import metrics
    from oracle import stap as orc
    acc = {}
    if len(wls) == 1:
        w = wls[0]
        N = w.n_cell
        errs, sls, pes = [], [], []
        for b in acc_blocks:
            ob = orc.run_block(cubes_np[0][:, :, b * N:(b + 1) * N], steers_np[0], w.tdof, w.load_eps)
            Wb = out_w[b]
            errs.append(metrics.rel_err(Wb, ob["W"][:, 0]))
            sls.append(float(metrics.sinr_loss_db(Wb, ob["W"][:, 0], steers_np[0], ob["R_L"][:, 0]).max()))
            pes.append(metrics.rel_err(out_power[b], ob["power"]))
        acc = dict(blocks=len(acc_blocks), weights_rel_err=max(errs), sinr_loss_db_max=max(sls),
                   power_rel_err=max(pes), info_nonzero=info_nonzero)

    cpu = None
    if not args.no_cpu and len(wls) == 1:
        w = wls[0]
        N = w.n_cell
        try:
            from threadpoolctl import threadpool_info
            threads = max([int(x.get("num_threads", 1)) for x in threadpool_info()] or [1])
        except Exception:
            threads = os.cpu_count()
        nb, t = 0, time.perf_counter()
        while True:
            b = (nb * 37) % w.n_block
            orc.run_block(cubes_np[0][:, :, b * N:(b + 1) * N], steers_np[0], w.tdof, w.load_eps)
            nb += 1
            el = time.perf_counter() - t
            if (el > args.cpu_seconds and nb >= 2) or nb >= w.n_block:
                break
        cpu = dict(value=nb * N * w.dof / el, unit="range-cell*DOF/s", cores=threads, kind="oracle",
                   sample=f"{nb} training blocks of {N} cells x all {w.n_pulse} bins (oracle.run_block), "
                          f"{el:.1f} s; host os.cpu_count()={os.cpu_count()}")
        # the same oracle on one thread (the analogue of sequential NumPy)
        try:
            from threadpoolctl import threadpool_limits
            with threadpool_limits(limits=1):
                nb1, t1 = 0, time.perf_counter()
                while True:
                    b = (nb1 * 53 + 11) % w.n_block
                    orc.run_block(cubes_np[0][:, :, b * N:(b + 1) * N], steers_np[0], w.tdof, w.load_eps)
                    nb1 += 1
                    el1 = time.perf_counter() - t1
                    if (el1 > args.cpu_seconds_single and nb1 >= 1) or nb1 >= w.n_block:
                        break
            cpu["single_thread"] = dict(value=nb1 * N * w.dof / el1, cores=1,
                                        sample=f"{nb1} training blocks, {el1:.1f} s, BLAS limited to one thread")
        except ImportError:
            pass

    # the paper's own cube (100 pulses x 1000 channels x 30000 samples, stored
    # pulses x channels x samples), 1000 elements in 20 subarrays (D = 60):
    # one stap_run per cube, resident in HBM; values are device-generated
    # complex Gaussian noise (the kernels' time does not depend on them)
    paper = None
    if not args.no_paper and len(wls) == 1:
        del cubes
        torch.cuda.empty_cache()
        wp = synth.PAPER
        g = torch.Generator(device=dev)
        g.manual_seed(wp.seed)
        pcube = torch.randn((wp.n_pulse, wp.n_chan, wp.n_range), dtype=torch.complex64, device=dev, generator=g)
        pv = torch.from_numpy(synth.steering(wp)).to(dev)
        pprob = stap.problem(wp.n_chan, wp.n_pulse, wp.n_range, wp.tdof, wp.n_block, wp.n_steer,
                             load_eps=wp.load_eps, precision=args.precision, refine_steps=args.refine,
                             cube_stride_chan=wp.n_range, cube_stride_pulse=wp.n_chan * wp.n_range, n_sub=wp.n_sub)
        prun = stap.Runner([pprob], device=dev)
        ppow = [torch.empty((wp.n_pulse, wp.n_steer, wp.n_range), dtype=torch.float32, device=dev)]
        for _ in range(2):
            prun.run([pcube], [pv], powers=ppow)
        torch.cuda.synchronize()
        psteps = 5
        t = time.perf_counter()
        for _ in range(psteps):
            prun.run([pcube], [pv], powers=ppow)
        torch.cuda.synchronize()
        pms = (time.perf_counter() - t) / psteps * 1e3
        # host-to-device rate from pinned memory, for the rate of a cube that
        # starts in host memory (copies overlapped with the previous cube's
        # processing, the PCIe-inclusive rate is the smaller of the two)
        hbuf = torch.empty(1 << 30, dtype=torch.uint8, pin_memory=True)
        dbuf = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dbuf.copy_(hbuf, non_blocking=True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(3):
            dbuf.copy_(hbuf, non_blocking=True)
        torch.cuda.synchronize()
        h2d = 3 * (1 << 30) / (time.perf_counter() - t)
        del hbuf, dbuf
        cube_bytes = wp.n_pulse * wp.n_chan * wp.n_range * 8
        paper = dict(workload=wp.name, layout="pulses x channels x samples (strides)", subarray=wp.n_sub,
                     h2d_GBps=h2d / 1e9,
                     pcie_inclusive_cubes_per_s=min(1e3 / pms, h2d / cube_bytes),
                     D=wp.dof, B=wp.n_block, N=wp.n_cell, S=wp.n_steer, precision=args.precision,
                     refine_steps=args.refine, ms_per_cube=pms, cubes_per_s=1e3 / pms,
                     real_time_cubes_per_s=33.3, value=wp.cells_dof / (pms * 1e-3), steps=psteps,
                     cube_gb=wp.n_pulse * wp.n_chan * wp.n_range * 8 / 1e9,
                     data="device-generated CN(0,1) noise of the cube's shape")
        del pcube, ppow, prun
        torch.cuda.empty_cache()

    name = args.workload if len(wls) > 1 else wls[0].name
    value = cells_dof / wall_m
    line = {
        "metric": "range-cell*DOF/s per datacube, mixed vs plain FP32 at <=0.1 dB SINR loss",
        "value": value,
        "unit": "range-cell*DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall_m * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": name, "cubes": len(wls), "precision": args.precision,
                   "refine_steps": args.refine,
                   **({} if len(wls) > 1 else dict(C=wls[0].n_chan, P=wls[0].n_pulse, R=wls[0].n_range,
                                                   D=wls[0].dof, B=wls[0].n_block, N=wls[0].n_cell,
                                                   S=wls[0].n_steer))},
        "event_ms_per_step": ev_m,
        "plain_fp32": plain,
        "mixed_over_plain": (value / plain["value"]) if plain else None,
        "mixed_without_refinement": unrefined,
        "accuracy": acc,
        "kernels": kern,
        "roofline": roof,
        "cpu_baseline": cpu,
        "paper_cube": paper,
        "gen_seconds": gen_s,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
