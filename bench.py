"""Benchmark: predict+gradient visibilities per second on one MI355X.

One step is one pass of the hot path over the whole workload: kernel
construction, degridding of V^M and its four offset derivatives, residual,
float64 per-antenna chi^2 / gradient / normal-matrix sums (psc_gradient), and
the damped per-antenna update (psc_solve_step).  The default workload is the
single-interval configuration: 27 antennas in a Y (351 baselines, arms to
21 km), 360 x 10 s, 16 channels over 1-2 GHz, one polarisation, a 1024^2
model grid with 200 point sources, support 16, oversampling 4.

Prints one JSON line (see the repository's benchmark contract).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK = 157.3e12  # MI355X published FP32 vector rate (FLOP/s)
HBM_PEAK = 8.0e12


KERNEL_SOURCES = ("psc_kernels.hip", "psc_device.h", "psc_internal.h")


def kernel_source_hash():
    """sha256 (first 16 hex digits) over the sources the table-form kernel is
    built from."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1709_08681_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the gradient kernel from the committed rocprofv3
    summary, or None when the kernel sources have changed since it was taken."""
    import re
    prof = os.path.join(ROOT, "profiles", "k_item_grad_single_interval.md")
    try:
        h = kernel_source_hash()
        txt = open(prof).read()
    except OSError:
        return None
    m = re.search(r"traffic_bytes=(\d+) kernel_source_sha256_16=([0-9a-f]+)", txt)
    return int(m.group(1)) if m and m.group(2) == h else None


def describe(obs):
    wl = obs.wl
    return {
        "workload": f"{wl.name}: {obs.n_ant} antennas ({wl.layout}), {wl.n_bl} baselines, "
                    f"{wl.n_time} x {wl.dt_s:g} s, {obs.n_chan} channels, {obs.n_pol} pol, "
                    f"{obs.n_int} interval(s), {obs.grid_n}^2 grid, support {wl.support}, "
                    f"oversampling {wl.oversample}",
        "n_vis": int(obs.n_vis),
        "n_intervals": int(obs.n_int),
        "grid_n": int(obs.grid_n),
        "support": int(wl.support),
        "oversample": int(wl.oversample),
        "step": "psc_gradient + psc_solve_step",
    }


def batched_vs_plain(cfg, iters, device=0, **overrides):
    """Algorithm 1 over every solution interval of workload `cfg` for a fixed
    number of iterations (tol = 0), in the three execution forms: PLAIN (host
    loop over intervals, launches per interval, host check per iteration),
    BATCHED (every interval in one launch set per iteration) and GRAPH
    (BATCHED, all iterations captured in one HIP graph and replayed).
    `overrides` change the workload (e.g. its interval lengths)."""
    import torch
    from paper_1709_08681_amd import synth
    from paper_1709_08681_amd import psc as P
    obs = synth.make_config(cfg, **overrides)
    s = P.Session(obs, device=device)
    try:
        v_obs = s.predict(s.offsets(obs.offsets_true))
        w = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
        start = s.offsets(synth.perturbed_offsets(obs, 30.0, 98))
        # the autotuner keeps the fastest degrid variant for all three forms
        tune_us = P.psc_tune(s.ctx, s.handle, start, v_obs, w, 2, None)
        variant = P.psc_get_degrid(s.handle)
        res = {}
        for name, form in (("plain", P.SOLVE_PLAIN), ("batched", P.SOLVE_BATCHED),
                           ("graph", P.SOLVE_GRAPH)):
            off = start.clone()
            s.solve(v_obs, w, off, gain=0.5, n_max=1, tol_rad=0.0, form=form)  # warm-up
            off = start.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.solve(v_obs, w, off, gain=0.5, n_max=iters, tol_rad=0.0, form=form)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            res[name] = {"vis_per_s": obs.n_vis * iters / dt, "ms_per_iteration": dt * 1e3 / iters}
            res[name + "_offsets"] = off
        same = bool(torch.equal(res["plain_offsets"], res["graph_offsets"]) and
                    torch.equal(res["batched_offsets"], res["graph_offsets"]))
        out = {k: v for k, v in res.items() if not k.endswith("_offsets")}
        out.update({
            "workload": describe(obs)["workload"],
            "n_vis": int(obs.n_vis),
            "iterations": iters,
            "graph_over_plain": out["graph"]["vis_per_s"] / out["plain"]["vis_per_s"],
            "bit_identical_offsets": same,
            "degrid": {P.DEGRID_VALU: "table, vector", P.DEGRID_MFMA: "table, matrix cores",
                       P.DEGRID_WINDOW: "window"}[variant],
            "tune_us": {"vector": tune_us[0], "matrix_core": tune_us[1], "window": tune_us[2]},
        })
        return out
    finally:
        s.close()


def image_gradient_timing(s, obs, off, v_obs, w, reps, stream):
    """psc_image_gradient (d chi^2 / d I on the model grid) on the same data:
    predict, residual scatter through per-item LDS patches (float64 atomics
    once per patch cell), float64 N^2 FFT."""
    import torch
    from paper_1709_08681_amd import psc as P
    n = obs.grid_n
    out = torch.empty((n, n), dtype=torch.float64, device=s.dev)
    P.psc_image_gradient(s.ctx, s.handle, off, v_obs, w, out, None, stream)  # warm-up, scratch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        P.psc_image_gradient(s.ctx, s.handle, off, v_obs, w, out, None, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"ms_per_call": ms, "vis_per_s": obs.n_vis / (ms * 1e-3), "calls": reps,
            "grid": f"{n}^2", "note": "table form, support 16, LDS-patch scatter"}


def extension_timing(obs, start, reps, what, device=0):
    """Gradient launches of one extension on the workload's data, on a session
    of its own:
      mount_frame        offsets in the antenna mount frame (every row's
                         parallactic angle), per-sample image-plane products;
      measured_aperture  the same with a measured, non-circular aperture
                         (bicubic lookups of its transform);
      measured_aperture_sky  the aperture without parallactic angles (its
                         products stored per item, five plain sums);
      beam_scale         psc_scale_gradient: the sums for a beam-width scale
                         per antenna (scales set within 3% of nominal);
      w_term             the workload's array shrunk to arms of 1 km (the
                         w-term's support limit; see the header), window form
                         with e^{2 pi i w (n-1)} per image sample."""
    import torch
    from paper_1709_08681_amd import psc as P
    from paper_1709_08681_amd import synth
    kw, note = {}, ""
    if what == "mount_frame":
        kw, note = dict(mount_frame=True), "window form, per-sample image-plane products"
    elif what == "measured_aperture":
        kw = dict(mount_frame=True, aperture=synth.measured_aperture())
        note = "window form, per-sample bicubic lookups of the aperture's transform, mount frame"
    elif what == "measured_aperture_sky":
        kw = dict(aperture=synth.measured_aperture())
        note = "window form, the aperture's products stored per item, sky frame"
    elif what == "beam_scale":
        kw, note = dict(mount_frame=True), "psc_scale_gradient, window form, mount frame"
    elif what == "w_term":
        if obs.wl.name != "single_interval":
            return {"skipped": "timed on the single-interval array only"}
        obs = synth.make_config(2, layout_radius_m=1000.0)
        start = synth.perturbed_offsets(obs, 30.0, 1)
        kw, note = dict(w_term=True), "window form with the w phase, arms shrunk to 1 km"
    s = P.Session(obs, device=device, **kw)
    try:
        stream = torch.cuda.current_stream()
        v = s.predict(s.offsets(obs.offsets_true))
        w = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
        off = s.offsets(start)
        if what == "beam_scale":
            s.set_beam_scale(np.random.default_rng(0).uniform(0.97, 1.03, s.off_shape[:3]))
            acc = torch.empty(s.off_shape[:3] + (3,), dtype=torch.float64, device=s.dev)
            call = lambda: P.psc_scale_gradient(s.ctx, s.handle, off, v, w, acc, stream)
        else:
            if what == "w_term":
                P.psc_set_degrid(s.handle, P.DEGRID_WINDOW)
            acc = torch.empty(s.off_shape[:3] + (6,), dtype=torch.float64, device=s.dev)
            call = lambda: P.psc_gradient(s.ctx, s.handle, off, v, w, acc, None, stream)
        call()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            call()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res = {"ms_per_gradient": ms, "vis_per_s": obs.n_vis / (ms * 1e-3), "calls": reps, "note": note}
        if what == "mount_frame":
            pa = obs.par_angle
            res["par_angle_range_deg"] = [float(np.degrees(pa.min())), float(np.degrees(pa.max()))]
        return res
    finally:
        s.close()


def cpu_baseline(obs, start, seconds):
    """The oracle (FP64 direct sum) on the host cores: gradient + update
    iterations for about `seconds`, over the whole workload or, when one
    iteration would take far longer, over its first timesteps."""
    import oracle
    n_src = len(obs.src_flux) + (0 if obs.extra_flux is None else len(obs.extra_flux))
    budget = 5e8  # visibility x pixel terms, about 10 s of the oracle on 16 cores
    if obs.n_vis * n_src > budget:
        per_t = obs.n_vis / max(1, len(np.unique(obs.time_idx)))
        n_t = max(1, int(budget / (per_t * n_src)))
        obs = obs.subset(times=range(n_t))  # offsets keep their shape
    prob = oracle.Problem.from_observation(obs)
    v_obs_np = oracle.predict(prob, obs.offsets_true)  # untimed: the oracle's own data
    off = start.copy()
    t0 = time.perf_counter()
    iters = 0
    while True:
        acc = oracle.gradient(prob, off, v_obs_np, 1.0)
        off, _, _ = oracle.solve_step(acc, 0.5, off)
        iters += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    out = {
        "value": obs.n_vis * iters / dt,
        "unit": "vis/s",
        "cores": int(oracle.num_threads()),
        "kind": "oracle",
        "sample": f"{obs.n_vis} visibilities x {len(prob.src_flux)} sky pixels "
                  f"({'whole workload' if obs.n_vis * n_src <= budget else 'first timesteps'}), "
                  f"{iters} gradient+update iteration(s) in {dt:.1f} s, FP64 direct summation",
        "cpu_model": cpu_model(),
    }
    out.update(single_thread_rate(prob, off, v_obs_np))
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def single_thread_rate(prob, off, v_obs):
    """One gradient + update of the oracle on one thread, over the first
    rows of the same problem (a child process with OMP_NUM_THREADS=1; it
    does not touch the GPU)."""
    import subprocess
    import tempfile
    rows = int(min(prob.n_row, max(1, 2e7 // max(1, len(prob.src_flux) * prob.n_chan * prob.n_pol))))
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "sample.npz")
        np.savez(path, src_l=prob.src_l, src_m=prob.src_m, src_flux=prob.src_flux, ant1=prob.ant1[:rows],
                 ant2=prob.ant2[:rows], uv_m=prob.uv_m[:rows], freq_hz=prob.freq_hz,
                 offsets=np.ascontiguousarray(off[:1]), vis=np.ascontiguousarray(v_obs[:rows]),
                 scalars=np.array([prob.n_ant, prob.n_pol, prob._s.dish_diam_m, prob._s.squint_frac,
                                   prob._s.snap_scale]))
        code = (
            "import sys, time, numpy as np\n"
            f"sys.path.insert(0, {ROOT!r})\n"
            "import oracle\n"
            f"z = np.load({path!r})\n"
            "n_ant, n_pol, dish, squint, snap = z['scalars']\n"
            "p = oracle.Problem(z['src_l'], z['src_m'], z['src_flux'], int(n_ant), z['ant1'], z['ant2'], z['uv_m'],\n"
            "                   [0, len(z['ant1'])], z['freq_hz'], n_pol=int(n_pol), dish_diam_m=dish,\n"
            "                   squint_frac=squint, snap_scale=snap)\n"
            "t0 = time.perf_counter()\n"
            "acc = oracle.gradient(p, z['offsets'], z['vis'], 1.0)\n"
            "oracle.solve_step(acc, 0.5, z['offsets'])\n"
            "print(time.perf_counter() - t0, oracle.num_threads())\n")
        env = dict(os.environ, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    if r.returncode != 0:
        return {"single_thread": f"failed: {r.stderr.strip()[-200:]}"}
    dt, nthr = r.stdout.split()[-2:]
    n = rows * prob.n_chan * prob.n_pol
    return {"single_thread_vis_per_s": n / float(dt),
            "single_thread_sample": f"{n} visibilities (first {rows} rows, one interval), "
                                    f"{int(nthr)} thread, one gradient+update in {float(dt):.2f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--channels", type=int, default=0,
                    help="keep the first N channels: one GPU's channel share of a larger workload")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched-config", type=int, default=3)
    ap.add_argument("--batched-iters", type=int, default=3)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-image-gradient", action="store_true")
    ap.add_argument("--no-mount-frame", action="store_true")
    ap.add_argument("--no-extensions", action="store_true",
                    help="skip the measured-aperture, beam-scale and w-term timings")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on one GPU only; sharding the path across GPUs (by solution "
              "interval or by channel block) is designed but not implemented.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1709_08681_amd import synth
    from paper_1709_08681_amd import psc as P
    from paper_1709_08681_amd.psc import Session, psc_gradient, psc_solve_step

    obs = synth.make_config(args.config)
    if args.channels:
        obs = obs.subset(chans=range(args.channels))
    print(f"bench: workload {obs.wl.name}, {obs.n_vis} visibilities", file=sys.stderr, flush=True)
    s = Session(obs, device=0)
    stream = torch.cuda.current_stream()
    off_true = s.offsets(obs.offsets_true)
    v_obs = s.predict(off_true)
    w = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
    start = synth.perturbed_offsets(obs, 30.0, 99)
    off = s.offsets(start)
    acc = torch.empty(s.off_shape[:3] + (6,), dtype=torch.float64, device=s.dev)
    mx = torch.empty(obs.n_int, dtype=torch.float64, device=s.dev)
    # the autotuner times every degrid variant on this data and keeps the fastest
    tune_us = P.psc_tune(s.ctx, s.handle, off, v_obs, w, 3, stream)
    variant = P.psc_get_degrid(s.handle)
    S = obs.wl.support
    kernel = {P.DEGRID_VALU: f"k_item<{S},grad> (table form, vector FP32)",
              P.DEGRID_MFMA: f"k_item<{S},grad> (table form, FP32 matrix cores)",
              P.DEGRID_WINDOW: f"k_winw<{S},grad> (window form, {2 * S}-lane workers)"}[variant]

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        psc_gradient(s.ctx, s.handle, off, v_obs, w, acc, None, stream)
        if ev is not None:
            ev[1].record(stream)
        psc_solve_step(s.ctx, obs.n_int, obs.n_pol, obs.n_ant, acc, 0.5, 0.0, off, None, mx, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for k in range(args.steps):
        step(evs[k])
    t_end.record(stream)
    torch.cuda.synchronize()
    ms_total = t_start.elapsed_time(t_end)
    ms_step = ms_total / args.steps
    grad_ms = sum(a.elapsed_time(b) for a, b in evs) / args.steps
    value = obs.n_vis / (ms_step * 1e-3)

    flops = obs.n_vis * 40.0 * S * S  # five complex multiply-adds per tap
    achieved = flops / (grad_ms * 1e-3)
    roof = {
        "bound": "alu",
        "achieved": achieved / 1e12,
        "peak": FP32_VECTOR_PEAK / 1e12,
        "unit": "TFLOP/s",
        "frac": achieved / FP32_VECTOR_PEAK,
        "traffic": measured_traffic() if (args.config == 2 and variant == P.DEGRID_VALU) else None,
        "traffic_unit": "bytes per launch (FETCH_SIZE x2 + WRITE_SIZE, copy-calibrated)",
        "kernel": kernel + " + k_reduce",
        "launch_ms": grad_ms,
    }
    out = {
        "metric": "predict+gradient visibilities/s",
        "value": value,
        "unit": "vis/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "accumulate_dtype": "f64",
        "data": "synthetic",
        "config": dict(describe(obs), degrid=kernel,
                       tune_us={name: t for name, t in zip(("vector", "matrix_core", "window"), tune_us)}),
        "roofline": roof,
    }
    if not args.no_image_gradient and S == 16:
        print("bench: image gradient", file=sys.stderr, flush=True)
        out["image_gradient"] = image_gradient_timing(s, obs, off, v_obs, w, 5, stream)
    s.close()
    if not args.no_mount_frame:
        print("bench: mount-frame offsets", file=sys.stderr, flush=True)
        out["mount_frame"] = extension_timing(obs, start, 3, "mount_frame")
    if not args.no_extensions:
        out["extensions"] = {}
        for what in ("measured_aperture", "measured_aperture_sky", "beam_scale", "w_term"):
            print(f"bench: {what}", file=sys.stderr, flush=True)
            out["extensions"][what] = extension_timing(obs, start, 3, what)
    if not args.no_batched:
        print(f"bench: batched vs plain on workload {args.batched_config}", file=sys.stderr,
              flush=True)
        out["batched_vs_plain"] = batched_vs_plain(args.batched_config, args.batched_iters)
        # the same array with 1024 short intervals (1 to 8 timesteps): per-interval
        # launches then carry little work each
        short = [int(x) for x in np.random.default_rng(7).integers(1, 9, size=1024)]
        print("bench: batched vs plain, short intervals", file=sys.stderr, flush=True)
        out["batched_vs_plain_short"] = batched_vs_plain(args.batched_config, args.batched_iters,
                                                         interval_lengths=short)
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(obs, start, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
