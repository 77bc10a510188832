"""Benchmark: predict+gradient visibilities per second on one MI355X.

One step is one pass of the hot path over the whole workload: Algorithm 1's
body for every solution interval at once -- kernel construction, degridding
of V^M and its four offset derivatives, residual, float64 per-antenna chi^2 /
gradient / normal-matrix sums, and the damped per-antenna update with its
termination flags.

The headline workload is the batched configuration: 27 antennas in a Y (351
baselines, arms to 21 km), 256 solution intervals of 10 to 120 timesteps of
10 s (16,565 timesteps), 16 channels over 1-2 GHz, one polarisation, a 2048^2
model grid with 200 point sources, support 16, oversampling 4: 93,029,040
visibilities per step.  Steps run in the graph form (psc_solve, every
interval in one launch set per iteration, the K timed iterations captured
in one HIP graph and replayed); the plain form (a host loop over intervals
with per-interval launches) and the batched form without the graph are timed
beside it on the same data, and their offsets must agree bit for bit.

Prints one JSON line (see the repository's benchmark contract).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK = 157.3e12  # MI355X published FP32 vector rate (FLOP/s)
HBM_PEAK = 8.0e12

# committed rocprofv3 summaries: (file, sources the profiled kernel is built from)
PROFILES = {
    "window": ("k_winw_grad_batched.md", ("psc_window.hip", "psc_device.h", "psc_internal.h")),
    "table": ("k_item_grad_single_interval.md", ("psc_kernels.hip", "psc_device.h", "psc_internal.h")),
    "window_large": ("k_winw_grad_large_share.md", ("psc_window.hip", "psc_device.h", "psc_internal.h")),
}


def source_hash(sources):
    """sha256 (first 16 hex digits) over the kernel sources."""
    import hashlib
    h = hashlib.sha256()
    for name in sources:
        with open(os.path.join(ROOT, "paper_1709_08681_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(which):
    """HBM bytes per launch of a kernel from its committed rocprofv3 summary,
    or None when the kernel's sources have changed since it was taken."""
    import re
    name, sources = PROFILES[which]
    try:
        txt = open(os.path.join(ROOT, "profiles", name)).read()
        h = source_hash(sources)
    except OSError:
        return None
    m = re.search(r"traffic_bytes=(\d+) kernel_source_sha256_16=([0-9a-f]+)", txt)
    return int(m.group(1)) if m and m.group(2) == h else None


def describe(obs):
    wl = obs.wl
    return (f"{wl.name}: {obs.n_ant} antennas ({wl.layout}), {wl.n_bl} baselines, "
            f"{len(np.unique(obs.time_idx))} x {wl.dt_s:g} s, {obs.n_chan} channels, {obs.n_pol} pol, "
            f"{obs.n_int} interval(s), {obs.grid_n}^2 grid, support {wl.support}, "
            f"oversampling {wl.oversample}")


def kernel_name(P, variant, S, waves):
    return {P.DEGRID_VALU: f"k_item<{S},grad> (table form, vector FP32)",
            P.DEGRID_MFMA: f"k_item<{S},grad> (table form, FP32 matrix cores)",
            P.DEGRID_WINDOW: f"k_winw<{S},grad,{waves} waves> (window form, {2 * S}-lane workers)"}[variant]


def roofline(flops, kernel_ms, traffic, kernel):
    achieved = flops / (kernel_ms * 1e-3)
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": FP32_VECTOR_PEAK / 1e12,
            "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK, "traffic": traffic,
            "traffic_unit": "bytes per launch (FETCH_SIZE x2 + WRITE_SIZE, copy-calibrated)",
            "kernel": kernel + " + k_reduce", "launch_ms": kernel_ms}


class Workload:
    """A planned workload on the GPU: observed data made by psc_predict at the
    injected offsets, unit weights, a start 30 arcsec off per axis, the
    autotuner's degrid variant."""

    def __init__(self, cfg, channels=0, tune=True, **overrides):
        import torch
        from paper_1709_08681_amd import synth
        from paper_1709_08681_amd import psc as P
        self.torch, self.P = torch, P
        obs = synth.make_config(cfg, **overrides)
        if channels:
            obs = obs.subset(chans=range(channels))
        self.obs = obs
        self.s = P.Session(obs, device=0)
        s = self.s
        self.stream = torch.cuda.current_stream()
        self.v_obs = s.predict(s.offsets(obs.offsets_true))
        self.w = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
        self.start_np = synth.perturbed_offsets(obs, 30.0, 99)
        self.start = s.offsets(self.start_np)
        self.off = self.start.clone()  # one offsets buffer for every timed run
        self.acc = torch.empty(s.off_shape[:3] + (6,), dtype=torch.float64, device=s.dev)
        self.mx = torch.empty(obs.n_int, dtype=torch.float64, device=s.dev)
        self.tune_us = None
        if tune:
            self.tune_us = P.psc_tune(s.ctx, s.handle, self.start, self.v_obs, self.w, 3, self.stream)
        self.info = P.psc_obs_launch_info(s.handle)
        S = obs.wl.support
        self.kernel = kernel_name(P, self.info["degrid"], S, self.info["window_waves"])
        self.flops = obs.n_vis * 40.0 * S * S  # five complex multiply-adds per tap

    def solve_form(self, form, iters, warmup):
        """Algorithm 1 for `iters` iterations (tol = 0, so every interval runs
        them all) from the same start in the given form; returns (ms per
        iteration, offsets).  The warm-up call has the same arguments, so the
        graph form captures its graph there and the timed call only replays
        it."""
        torch, s = self.torch, self.s
        for k in range(max(1, warmup)):
            self.off.copy_(self.start)
            s.solve(self.v_obs, self.w, self.off, gain=0.5, n_max=iters, tol_rad=0.0, form=form)
        self.off.copy_(self.start)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.solve(self.v_obs, self.w, self.off, gain=0.5, n_max=iters, tol_rad=0.0, form=form)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return dt * 1e3 / iters, self.off.clone()

    def eager_steps(self, steps, warmup):
        """The same iteration written out with the C-ABI calls on the bench's
        stream (psc_gradient, then psc_solve_step), HIP events around every
        gradient launch: returns (ms per step, ms per gradient launch)."""
        torch, P, s, obs = self.torch, self.P, self.s, self.obs

        def step(ev=None):
            if ev is not None:
                ev[0].record(self.stream)
            P.psc_gradient(s.ctx, s.handle, self.off, self.v_obs, self.w, self.acc, None, self.stream)
            if ev is not None:
                ev[1].record(self.stream)
            P.psc_solve_step(s.ctx, obs.n_int, obs.n_pol, obs.n_ant, self.acc, 0.5, 0.0, self.off, None,
                             self.mx, self.stream)

        self.off.copy_(self.start)
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record(self.stream)
        for k in range(steps):
            step(evs[k])
        t1.record(self.stream)
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / steps, sum(a.elapsed_time(b) for a, b in evs) / steps

    def close(self):
        self.s.close()


def forms_report(wl, iters, warmup, forms=("graph", "batched", "plain")):
    """The three execution forms of Algorithm 1 on one workload."""
    P = wl.P
    code = {"plain": P.SOLVE_PLAIN, "batched": P.SOLVE_BATCHED, "graph": P.SOLVE_GRAPH}
    res, offs = {}, {}
    for name in forms:
        ms, offs[name] = wl.solve_form(code[name], iters, warmup)
        res[name] = {"vis_per_s": wl.obs.n_vis / (ms * 1e-3), "ms_per_iteration": ms}
        if name == "graph":
            # host time the library spent capturing and instantiating the
            # graph in the warm-up call (outside the timed call)
            res[name]["capture_and_instantiate_ms"] = P.psc_obs_launch_info(wl.s.handle)["capture_ms"]
    ref = offs[forms[0]]
    res["bit_identical_offsets"] = bool(all(wl.torch.equal(ref, o) for o in offs.values()))
    if "plain" in res and "graph" in res:
        res["graph_over_plain"] = res["graph"]["vis_per_s"] / res["plain"]["vis_per_s"]
    if "plain" in res and "batched" in res:
        res["batched_over_plain"] = res["batched"]["vis_per_s"] / res["plain"]["vis_per_s"]
    res["iterations"] = iters
    return res


def single_interval_extra(steps, warmup):
    """The single-interval workload (2,021,760 visibilities, 1024^2 grid): the
    eager step with its own roofline."""
    wl = Workload(2)
    try:
        ms_step, kern_ms = wl.eager_steps(steps, warmup)
        table = wl.info["degrid"] == wl.P.DEGRID_VALU
        return {"workload": describe(wl.obs), "n_vis": int(wl.obs.n_vis), "ms_per_step": ms_step,
                "vis_per_s": wl.obs.n_vis / (ms_step * 1e-3), "degrid": wl.kernel,
                "plan_ms": wl.info["plan_ms"],
                "tune_us": dict(zip(("vector", "matrix_core", "window"), wl.tune_us)),
                "roofline": roofline(wl.flops, kern_ms, measured_traffic("table") if table else None,
                                     wl.kernel)}
    finally:
        wl.close()


def large_share_extra(channels, iters):
    """One GPU's channel share of the large workload (128 antennas, 8128
    baselines, 600 x 10 s, 2 pols with opposite squint, 64 uneven intervals,
    4096^2 grid, support 32, oversampling 8): the three solve forms, the eager
    step's roofline, and the autograd forward + backward (psc_predict, then
    psc_predict_vjp through torch.autograd)."""
    torch = __import__("torch")
    from paper_1709_08681_amd.autograd import predict as diff_predict
    t0 = time.perf_counter()
    wl = Workload(5, channels=channels, tune=False)
    setup_s = time.perf_counter() - t0
    try:
        out = {"workload": describe(wl.obs), "n_vis": int(wl.obs.n_vis), "degrid": wl.kernel,
               "plan_ms": wl.info["plan_ms"], "setup_s": setup_s}
        out.update(forms_report(wl, iters, 1))
        ms_step, kern_ms = wl.eager_steps(iters, 1)
        out["eager"] = {"ms_per_step": ms_step, "vis_per_s": wl.obs.n_vis / (ms_step * 1e-3)}
        out["roofline"] = roofline(wl.flops, kern_ms, measured_traffic("window_large"), wl.kernel)
        # autograd: chi^2 = sum w |V_obs - V(p)|^2, backward through the adjoint
        p = wl.start.clone().requires_grad_(True)
        for k in range(2):
            torch.cuda.synchronize()
            ta = time.perf_counter()
            v = diff_predict(p, wl.s)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            loss = ((wl.v_obs - v).abs() ** 2).sum()
            loss.backward()
            torch.cuda.synchronize()
            tc = time.perf_counter()
            p.grad = None
            del v, loss
        out["autograd"] = {"forward_ms": (tb - ta) * 1e3, "backward_ms": (tc - tb) * 1e3,
                           "note": "psc_predict forward; chi^2 in torch; backward = psc_predict_vjp "
                                   "(kernels rebuilt, not stored) + torch's elementwise grad"}
        return out
    finally:
        wl.close()


def image_gradient_timing(wl, reps):
    """psc_image_gradient (d chi^2 / d I on the model grid) on the same data."""
    torch, P, s = wl.torch, wl.P, wl.s
    n = wl.obs.grid_n
    out = torch.empty((n, n), dtype=torch.float64, device=s.dev)
    P.psc_image_gradient(s.ctx, s.handle, wl.start, wl.v_obs, wl.w, out, None, wl.stream)  # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(wl.stream)
    for _ in range(reps):
        P.psc_image_gradient(s.ctx, s.handle, wl.start, wl.v_obs, wl.w, out, None, wl.stream)
    e1.record(wl.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"ms_per_call": ms, "vis_per_s": wl.obs.n_vis / (ms * 1e-3), "calls": reps,
            "grid": f"{n}^2"}


def extension_timing(cfg, reps, what):
    """Gradient launches of one extension on a workload's data, on a session of
    its own:
      mount_frame        offsets in the antenna mount frame (every row's
                         parallactic angle), per-sample image-plane products;
      measured_aperture  the same with a measured, non-circular aperture
                         (bicubic lookups of its transform);
      measured_aperture_sky  the aperture without parallactic angles (its
                         products stored per item, five plain sums);
      beam_scale         psc_scale_gradient: the sums for a beam-width scale
                         per antenna (scales set within 3% of nominal);
      w_term             the array's arms shrunk to 1 km (one kernel holds
                         the w-term), window form with e^{2 pi i w (n-1)}
                         per image sample;
      w_stack            the array as configured (arms to 21 km) with its w:
                         w-stacked model grids, each sample's residual w in
                         its kernel;
      defocus            psc_defocus_gradient: the sums for an aperture
                         defocus per antenna (within 0.5 rad), complex
                         patterns of the uniform disc."""
    import torch
    from paper_1709_08681_amd import psc as P
    from paper_1709_08681_amd import synth
    obs = synth.make_config(cfg, layout_radius_m=1000.0) if what == "w_term" else synth.make_config(cfg)
    start = synth.perturbed_offsets(obs, 30.0, 99)
    kw = {"mount_frame": dict(mount_frame=True),
          "measured_aperture": dict(mount_frame=True, aperture=synth.measured_aperture()),
          "measured_aperture_sky": dict(aperture=synth.measured_aperture()),
          "beam_scale": dict(mount_frame=True),
          "w_term": dict(w_term=True),
          "w_stack": dict(w_term=True),
          "defocus": {}}[what]
    s = P.Session(obs, device=0, **kw)
    try:
        stream = torch.cuda.current_stream()
        v = s.predict(s.offsets(obs.offsets_true))
        w = torch.ones(s.vis_shape, dtype=torch.float32, device=s.dev)
        off = s.offsets(start)
        if what == "beam_scale":
            s.set_beam_scale(np.random.default_rng(0).uniform(0.97, 1.03, s.off_shape[:3]))
            acc = torch.empty(s.off_shape[:3] + (3,), dtype=torch.float64, device=s.dev)
            call = lambda: P.psc_scale_gradient(s.ctx, s.handle, off, v, w, acc, stream)
        elif what == "defocus":
            s.set_defocus(np.random.default_rng(0).uniform(-0.5, 0.5, s.off_shape[:3]))
            acc = torch.empty(s.off_shape[:3] + (3,), dtype=torch.float64, device=s.dev)
            call = lambda: P.psc_defocus_gradient(s.ctx, s.handle, off, v, w, acc, stream)
        else:
            if what in ("w_term", "w_stack"):
                P.psc_set_degrid(s.handle, P.DEGRID_WINDOW)
            acc = torch.empty(s.off_shape[:3] + (6,), dtype=torch.float64, device=s.dev)
            call = lambda: P.psc_gradient(s.ctx, s.handle, off, v, w, acc, None, stream)
        call()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            call()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out = {"workload": describe(obs), "ms_per_gradient": ms, "vis_per_s": obs.n_vis / (ms * 1e-3),
               "calls": reps}
        if what == "w_stack":
            out["w_planes"] = P.psc_obs_launch_info(s.handle)["w_planes"]
        return out
    finally:
        s.close()


def cpu_baseline(cfg, start, seconds):
    """The oracle (FP64 direct sum, OpenMP on every host core) on a bounded
    sample of the workload: the first solution intervals whose visibilities
    times sky pixels stay within a budget of about ten seconds of oracle work
    per iteration, gradient + update iterations for about `seconds`.  The
    oracle's cost per visibility is proportional to the number of non-zero sky
    pixels, which the sample shares with the whole workload, so its vis/s
    stands for the whole workload's."""
    import oracle
    from paper_1709_08681_amd import synth
    obs = synth.make_config(cfg)
    n_src = len(obs.src_flux) + (0 if obs.extra_flux is None else len(obs.extra_flux))
    budget = 5e8  # visibility x pixel terms per iteration
    whole = obs.n_vis * n_src <= budget
    if not whole:
        per_row = obs.n_chan * obs.n_pol
        rows_ok = int(budget / (per_row * n_src))
        n_keep = int(np.searchsorted(obs.int_row_ptr, rows_ok, side="right")) - 1
        n_keep = max(1, n_keep)
        keep_t = np.unique(obs.time_idx[:obs.int_row_ptr[n_keep]])
        obs = obs.subset(times=keep_t)
    prob = oracle.Problem.from_observation(obs)
    v_obs_np = oracle.predict(prob, obs.offsets_true)  # untimed: the oracle's own data
    off = np.array(start, dtype=np.float64, copy=True)
    t0 = time.perf_counter()
    iters = 0
    while True:
        acc = oracle.gradient(prob, off, v_obs_np, 1.0)
        off, _, _ = oracle.solve_step(acc, 0.5, off)
        iters += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    live = int(np.count_nonzero(np.diff(obs.int_row_ptr)))
    out = {
        "value": obs.n_vis * iters / dt,
        "unit": "vis/s",
        "cores": int(oracle.num_threads()),
        "kind": "oracle",
        "sample": (f"{obs.n_vis} visibilities x {len(prob.src_flux)} sky pixels "
                   f"({'whole workload' if whole else f'the first {live} of {obs.n_int} solution intervals'}), "
                   f"{iters} gradient+update iteration(s) in {dt:.1f} s, FP64 direct summation"),
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
    """One gradient + update of the oracle on one thread, over the first rows
    of the same problem (a child process with OMP_NUM_THREADS=1; it does not
    touch the GPU)."""
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
    ap.add_argument("--config", type=int, default=3, help="headline workload (3: batched)")
    ap.add_argument("--channels", type=int, default=0,
                    help="keep the headline workload's first N channels (one GPU's channel share)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the single-interval, large-share, short-interval and extension timings")
    ap.add_argument("--large-channels", type=int, default=32,
                    help="channels of the large workload's share (one GPU of eight: 32)")
    ap.add_argument("--large-iters", type=int, default=2)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on one GPU only; sharding the path across GPUs (by solution "
              "interval or by channel block) is designed but not implemented.",
              file=sys.stderr)
        sys.exit(2)

    print(f"bench: headline workload {args.config}", file=sys.stderr, flush=True)
    wl = Workload(args.config, channels=args.channels, tune=True)
    obs = wl.obs
    rep = forms_report(wl, args.steps, args.warmup)
    ms_step = rep["graph"]["ms_per_iteration"]
    print("bench: eager steps with per-launch events", file=sys.stderr, flush=True)
    eager_ms, kern_ms = wl.eager_steps(args.steps, args.warmup)
    # the committed counters of this workload's kernel, when they are for it
    which = {(3, wl.P.DEGRID_WINDOW): "window", (2, wl.P.DEGRID_VALU): "table",
             (5, wl.P.DEGRID_WINDOW): "window_large"}.get((args.config, wl.info["degrid"]))
    traffic = measured_traffic(which) if which and (args.config != 5 or args.channels == 32) else None
    out = {
        "metric": "predict+gradient visibilities/s",
        "value": obs.n_vis / (ms_step * 1e-3),
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
        "config": {
            "workload": describe(obs),
            "n_vis": int(obs.n_vis),
            "n_intervals": int(obs.n_int),
            "grid_n": int(obs.grid_n),
            "support": int(obs.wl.support),
            "oversample": int(obs.wl.oversample),
            "step": "one Algorithm-1 iteration over every interval: psc_solve, graph form",
            "degrid": wl.kernel,
            "samples_per_item": wl.info["samples_per_item"],
            "plan_ms": wl.info["plan_ms"],
            "tune_us": dict(zip(("vector", "matrix_core", "window"), wl.tune_us)),
        },
        "roofline": roofline(wl.flops, kern_ms, traffic, wl.kernel),
        "batched_vs_plain": rep,
        "eager_step": {"ms_per_step": eager_ms, "ms_per_gradient_launch": kern_ms,
                       "note": "psc_gradient + psc_solve_step on the bench's stream, HIP events "
                               "around each gradient launch; the roofline's launch time"},
    }
    if not args.no_extras and obs.wl.support == 16:
        print("bench: image gradient", file=sys.stderr, flush=True)
        out["image_gradient"] = image_gradient_timing(wl, 3)
    wl.close()
    if not args.no_extras:
        print("bench: single interval", file=sys.stderr, flush=True)
        out["single_interval"] = single_interval_extra(args.steps, args.warmup)
        print("bench: short intervals", file=sys.stderr, flush=True)
        # the batched array with 1024 intervals of 1 to 8 timesteps: per-interval
        # launches then carry little work each
        short = [int(x) for x in np.random.default_rng(7).integers(1, 9, size=1024)]
        wls = Workload(3, interval_lengths=short)
        try:
            out["batched_vs_plain_short"] = dict(forms_report(wls, 3, 1), workload=describe(wls.obs),
                                                 n_vis=int(wls.obs.n_vis), degrid=wls.kernel)
        finally:
            wls.close()
        print(f"bench: large workload, {args.large_channels}-channel share", file=sys.stderr, flush=True)
        out["large_share"] = large_share_extra(args.large_channels, args.large_iters)
        out["extensions"] = {}
        for what in ("mount_frame", "measured_aperture", "measured_aperture_sky", "beam_scale", "w_term",
                     "w_stack", "defocus"):
            print(f"bench: {what}", file=sys.stderr, flush=True)
            out["extensions"][what] = extension_timing(2, 3, what)
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.config, wl.start_np, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
