"""Benchmark: 3DGS backward ms/iter, wave-reduce vs plain atomics, on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large_3m|object_100k]
                    [--no-object] [--no-batch] [--no-serve] [--no-cpu-baseline]

A step is one pass of the whole path over one synthetic view: render
(projection, binning with the device radix sort, forward composite), the
workload's loss gradient (L1 for the 3M-Gaussian 1080p view, L1 + 0.2 D-SSIM
for the object scene), and the backward (backward composite + per-Gaussian
chain rule), inputs already resident in HBM. The default view is the large
one: 3M Gaussians at 1920x1080 with the camera inside the cloud. `value` is
the backward's milliseconds per iteration (the whole backward call: clearing
the accumulator rows, backward composite, preprocess backward) in wave-reduce mode at the balancing threshold picked by a
one-iteration-per-candidate sweep (the paper's tuning rule); the
plain-atomic backward on the same forward state is reported beside it, as
are the atomic counts, both backward kernels against their roofs and the
fp64 oracle timed on the host cores. Further legs: the 100k-Gaussian 800x800
object view (A/B), the 16-view four-scene batch (autotuned, batched vs one
view at a time, hipGraph replay) and the served request stream (continuous
batching vs a sequential plain-atomic server, p50/p99 latency and steps/s at
several Poisson arrival rates).

Prints exactly one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

THRESHOLDS = [1, 2, 4, 8, 16, 24, 32, 48, 64]
PEAK_FP32_VALU_TFLOPS = 157.3     # MI355X fp32 vector peak (256 CUs x 2.4 GHz x 256 flop/clk)
PEAK_HBM_GBS = 8000.0
# Algorithmic fp32 work of the backward composite: per evaluated (pixel, entry) pair the splat
# evaluation (offset, quadratic form, exp), per contributing pair the transmittance division,
# colour update, dL/dalpha and the nine gradient values, per reduced wave-entry the nine values'
# six butterfly steps (12 E + 45 A + 54 W_R).
FLOPS_PER_EVAL = 12
FLOPS_PER_CONTRIB = 45
FLOPS_PER_REDUCED = 54
BYTES_PER_RECORD = 40             # id + mean2d + conic + opacity + rgb, read once per entry a tile's block walks
BYTES_PER_PIXEL = 20              # dL/dI (12) + T_final (4) + n_contrib (4)
BYTES_PER_VISIBLE = 72            # nine fp64 sums written back once (their clearing excluded; a7 reads them)


MODES = {"reduce": 1, "plain": 0, "serial": 2, "block": 3, "compiler": 4}   # gsr_bwd_mode values


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="large_3m", choices=["object_100k", "large_3m"])
    p.add_argument("--no-object", action="store_true", help="skip the 100k-Gaussian 800x800 A/B leg")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--threshold", type=int, default=None, help="fix the threshold (skip the sweep)")
    p.add_argument("--profile-only", action="store_true", help="only the timed steps (for rocprofv3 runs)")
    p.add_argument("--mode", default="reduce", choices=list(MODES), help="backward mode of --profile-only")
    p.add_argument("--no-lane-split", action="store_true",
                   help="reduced sums issued by one lane (default: nine lanes, one instruction)")
    p.add_argument("--no-batch", action="store_true", help="skip the 16-view batched leg")
    p.add_argument("--no-serve", action="store_true", help="skip the served request stream")
    p.add_argument("--profile-batch", default=None, metavar="TILE,LDS,THR",
                   help="only the 16-view batched render + backward at this fixed configuration, --steps "
                        "times (for rocprofv3 runs: no autotuning, no graph capture)")
    p.add_argument("--serve-seconds", type=float, default=1.5, help="seconds of arrivals per rate")
    p.add_argument("--serve-only", action="store_true", help="only the served request stream (its JSON)")
    p.add_argument("--xcd-remap", action="store_true", help="map neighbouring tiles to one XCD")
    p.add_argument("--no-tile-order", action="store_true", help="launch tiles in index order (no longest-first)")
    p.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                   help="only run a plain device copy of MIB MiB five times (reference for HBM counters)")
    p.add_argument("--microbench", default=None, metavar="KIND:MIB",
                   help="only run one library micro-benchmark (write, read, copy_nt, gather48) over MIB MiB, "
                        "one untimed and five timed launches (references of known bytes for HBM counters)")
    return p.parse_args()


def measure_roofs(ctx):
    """Copy bandwidth and atomic rates of the backward's access patterns (library micro-benchmarks)."""
    from paper_2401_05345_amd import gsr
    mib = 1 << 20

    def rate(kind, nbytes):
        ms, ops = gsr.gsr_microbench(ctx, kind, nbytes, reps=5)
        return ops / (ms * 1e-3)

    out = {"hbm_copy_GBs": round(rate(gsr.GSR_MB_COPY, 1024 * mib) / 1e9, 1),
           "hbm_copy_nt_GBs": round(rate(gsr.GSR_MB_COPY_NT, 1024 * mib) / 1e9, 1),
           "hbm_write_GBs": round(rate(gsr.GSR_MB_WRITE, 1024 * mib) / 1e9, 1),
           "hbm_read_GBs": round(rate(gsr.GSR_MB_READ, 1024 * mib) / 1e9, 1),
           "gather48_GBs": round(rate(gsr.GSR_MB_GATHER48, 1024 * mib) / 1e9, 1), "atomic_Gops": {}}
    for name, kind, nbytes in [("f32_distinct_2MiB", gsr.GSR_MB_ATOMIC_F32_DISTINCT, 2 * mib),
                               ("f32_distinct_128MiB", gsr.GSR_MB_ATOMIC_F32_DISTINCT, 128 * mib),
                               ("f64_distinct_128MiB", gsr.GSR_MB_ATOMIC_F64_DISTINCT, 128 * mib),
                               ("f32_same_address_16MiB", gsr.GSR_MB_ATOMIC_F32_SAME_ADDRESS, 16 * mib),
                               ("f32_one_lane_16MiB", gsr.GSR_MB_ATOMIC_F32_ONE_LANE, 16 * mib),
                               ("f64_nine_lanes_16MiB", gsr.GSR_MB_ATOMIC_F64_NINE_LANES, 16 * mib)]:
        out["atomic_Gops"][name] = round(rate(kind, nbytes) / 1e9, 3)
    log(f"[bench] roofs: {out}")
    return out


class Bench:
    def __init__(self, wl):
        import torch
        from paper_2401_05345_amd import gsr
        self.torch, self.gsr = torch, gsr
        self.wl = wl
        dev = torch.device("cuda:0")
        self.t = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in wl.scene.arrays()]
        self.scene = gsr.make_scene(*self.t, wl.scene.sh_degree)
        c = wl.camera
        self.cam = gsr.make_camera(c.width, c.height, c.fx, c.fy, c.cx, c.cy, c.world_to_cam, c.znear, c.bg)
        self.r = gsr.Renderer(0)
        self.grads = [torch.zeros_like(x) for x in self.t]
        self.gstruct = gsr.make_grads(*self.grads)
        self.dl = torch.empty((3, c.height, c.width), device=dev)
        # Target image: the render of the perturbed parameters (object scene) or the drawn target.
        if wl.perturbed is not None:
            tp = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in wl.perturbed.arrays()]
            fr = self.r.render(gsr.make_scene(*tp, wl.scene.sh_degree), self.cam, gsr.make_config())
            self.target = fr.image.clone()
            self.r.release(fr)
        else:
            self.target = torch.from_numpy(wl.target).to(dev)

    extra_flags = 0

    def cfg(self, mode, thr, flags=0):
        return self.gsr.make_config(16, 256, mode, thr, flags | self.extra_flags | self.gsr.GSR_FLAG_STAGE_TIMING)

    def step(self, cfg):
        """One whole pass; returns (stage times, frame stats)."""
        fr = self.r.render(self.scene, self.cam, cfg)
        self.loss_grad(fr.image)
        self.gsr.gsr_backward(self.r.ctx, fr.state, self.dl, self.gstruct, 0, cfg)
        st = self.gsr.gsr_ctx_stage_times(self.r.ctx)
        stats = fr.stats
        self.r.release(fr)
        return st, stats

    def backward_only(self, fr, cfg, iters, clear=None):
        """Backward repeated on one forward state; returns per-iteration (a6, a7) ms lists (and the
        ms of the accumulator clearing and tile ordering before a6 in `clear` when given)."""
        a6, a7 = [], []
        for _ in range(iters):
            self.gsr.gsr_backward(self.r.ctx, fr.state, self.dl, self.gstruct, 0, cfg)
            st = self.gsr.gsr_ctx_stage_times(self.r.ctx)
            a6.append(st.composite_bwd)
            a7.append(st.preprocess_bwd)
            if clear is not None:
                clear.append(st.zero_acc)
        return a6, a7

    def loss_grad(self, image):
        """dL/dimage of the workload's loss: L1, or L1 + 0.2 D-SSIM (object scene)."""
        if self.wl.loss == "l1_dssim":
            self.gsr.gsr_l1_dssim_grad(self.r.ctx, image, self.target, self.dl, 0.2)
        else:
            self.gsr.gsr_l1_grad(self.r.ctx, image, self.target, self.dl)

    def forward_state(self, cfg):
        fr = self.r.render(self.scene, self.cam, cfg)
        self.loss_grad(fr.image)
        return fr

    def sweep(self, fr, iters=3):
        gsr = self.gsr
        res = {}
        for thr in THRESHOLDS:
            a6, _ = self.backward_only(fr, self.cfg(gsr.GSR_BWD_WAVE_REDUCE, thr), iters)
            res[thr] = float(np.median(a6))
        return res

    def counters(self, fr, mode, thr):
        gsr = self.gsr
        cfg = gsr.make_config(16, 256, mode, thr, gsr.GSR_FLAG_DEBUG_COUNTERS | self.extra_flags)
        gsr.gsr_backward(self.r.ctx, fr.state, self.dl, self.gstruct, 0, cfg)
        return gsr.gsr_bwd_counters(self.r.ctx, fr.state)


def timed_ms(torch, fn, reps):
    """Median milliseconds of fn() between events on the current (null) stream."""
    out = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        out.append(a.elapsed_time(b))
    return float(np.median(out))


def bench_multi_view(flags, reps=5):
    """16 views of four scenes of uneven size at mixed resolutions: batched render and backward
    (one composite launch per pass over every (view, tile) pair) at the autotuned configuration,
    against the same views rendered and differentiated one call at a time; the batched backward
    also replayed from a captured hipGraph; the plain-atomic batched backward beside it."""
    import torch
    from paper_2401_05345_amd import gsr
    from paper_2401_05345_amd import scenegen as sg
    mv = sg.multi_view()
    log(f"[bench] {mv.name}: {[s.n for s in mv.scenes]} Gaussians, {len(mv.views)} views")
    dev = torch.device("cuda:0")
    st_t = [[torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in s.arrays()] for s in mv.scenes]
    structs = [gsr.make_scene(*t, s.sh_degree) for t, s in zip(st_t, mv.scenes)]
    grads_t = [[torch.zeros_like(x) for x in t] for t in st_t]
    gstructs = [gsr.make_grads(*g) for g in grads_t]
    scenes, cams, targets, imgs, dls, outs = [], [], [], [], [], []
    for si, c, tgt in mv.views:
        scenes.append(structs[si])
        cams.append(gsr.make_camera(c.width, c.height, c.fx, c.fy, c.cx, c.cy, c.world_to_cam, c.znear, c.bg))
        targets.append(torch.from_numpy(tgt).to(dev))
        imgs.append(torch.empty((3, c.height, c.width), device=dev))
        dls.append(torch.empty((3, c.height, c.width), device=dev))
        outs.append(gstructs[si])
    r = gsr.Renderer(0)
    ctx = r.ctx
    space = gsr.make_tune_space(reps=2, flags=flags)
    t0 = time.perf_counter()
    best, entries = gsr.gsr_autotune(ctx, scenes, cams, space)
    tune_s = time.perf_counter() - t0
    cfg = gsr.make_config(best.tile, best.lds_batch, gsr.GSR_BWD_WAVE_REDUCE, best.reduce_threshold, flags)
    cfg_plain = gsr.make_config(best.tile, best.lds_batch, gsr.GSR_BWD_PLAIN_ATOMIC, 0, flags | gsr.GSR_FLAG_ACC_F32)
    log(f"[bench] autotune ({tune_s:.1f} s): tile {best.tile}, lds {best.lds_batch}, thr {best.reduce_threshold}")

    states = gsr.gsr_render_batch(ctx, scenes, cams, cfg, imgs)
    for im, tg, d in zip(imgs, targets, dls):
        gsr.gsr_l1_grad(ctx, im, tg, d)
    res = {}

    def render_batch():
        for s in gsr.gsr_render_batch(ctx, scenes, cams, cfg, imgs):
            gsr.gsr_fwd_release(ctx, s)

    def render_seq():
        for sc, cm, im in zip(scenes, cams, imgs):
            gsr.gsr_fwd_release(ctx, gsr.gsr_render(ctx, sc, cm, cfg, im))

    def bwd_batch(c=cfg):
        gsr.gsr_backward_batch(ctx, states, dls, outs, 0, c)

    def bwd_seq():
        seen = set()
        for st, d, o, si in zip(states, dls, outs, [v[0] for v in mv.views]):
            gsr.gsr_backward(ctx, st, d, o, 1 if si in seen else 0, cfg)
            seen.add(si)

    for name, fn in (("render_batch_ms", render_batch), ("render_sequential_ms", render_seq),
                     ("backward_batch_ms", bwd_batch), ("backward_sequential_ms", bwd_seq),
                     ("backward_batch_plain_ms", lambda: bwd_batch(cfg_plain))):
        fn()
        res[name] = round(timed_ms(torch, fn, reps), 4)
    graph = gsr.gsr_graph_capture_backward(ctx, states, dls, outs, 0, cfg)
    gsr.gsr_graph_launch(ctx, graph)
    res["backward_graph_ms"] = round(timed_ms(torch, lambda: gsr.gsr_graph_launch(ctx, graph), reps), 4)
    gsr.gsr_graph_destroy(ctx, graph)
    pairs = [int(gsr.gsr_fwd_stats(s).n_pairs) for s in states]
    for s in states:
        gsr.gsr_fwd_release(ctx, s)
    r.close()
    tot = sorted(entries, key=lambda e: e.render_ms + e.backward_ms)
    res.update({
        "workload": mv.name, "n_views": len(mv.views), "gaussians": [s.n for s in mv.scenes],
        "resolutions": [[v[1].width, v[1].height] for v in mv.views], "n_pairs_total": sum(pairs),
        "autotune": {"tile": best.tile, "lds_batch": best.lds_batch, "threshold": best.reduce_threshold,
                     "seconds": round(tune_s, 2), "candidates": len(entries),
                     "best_ms": round(tot[0].render_ms + tot[0].backward_ms, 3),
                     "worst_ms": round(tot[-1].render_ms + tot[-1].backward_ms, 3),
                     "table": [[e.config.tile, e.config.lds_batch, e.config.reduce_threshold,
                                round(e.render_ms, 3), round(e.backward_ms, 3)] for e in entries]},
        "speedup_backward_batch_vs_sequential": round(res["backward_sequential_ms"] / res["backward_batch_ms"], 3),
        "speedup_render_batch_vs_sequential": round(res["render_sequential_ms"] / res["render_batch_ms"], 3),
        "speedup_backward_reduce_vs_plain": round(res["backward_batch_plain_ms"] / res["backward_batch_ms"], 3),
    })
    log(f"[bench] multi-view: {json.dumps({k: v for k, v in res.items() if k != 'autotune'})}")
    return res


def profile_multi_view(flags, spec, steps, warmup):
    """The 16-view batch's kernels alone: batched render, L1 gradient and batched backward at a
    fixed (tile, LDS batch, threshold), with no autotuner and no graph capture."""
    import torch
    from paper_2401_05345_amd import gsr
    from paper_2401_05345_amd import scenegen as sg
    tile, lds, thr = (int(x) for x in spec.split(","))
    mv = sg.multi_view()
    dev = torch.device("cuda:0")
    st_t = [[torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in s.arrays()] for s in mv.scenes]
    structs = [gsr.make_scene(*t, s.sh_degree) for t, s in zip(st_t, mv.scenes)]
    grads_t = [[torch.zeros_like(x) for x in t] for t in st_t]   # held: the structs keep bare pointers
    gstructs = [gsr.make_grads(*g) for g in grads_t]
    scenes, cams, targets, imgs, dls, outs = [], [], [], [], [], []
    for si, c, tgt in mv.views:
        scenes.append(structs[si])
        cams.append(gsr.make_camera(c.width, c.height, c.fx, c.fy, c.cx, c.cy, c.world_to_cam, c.znear, c.bg))
        targets.append(torch.from_numpy(tgt).to(dev))
        imgs.append(torch.empty((3, c.height, c.width), device=dev))
        dls.append(torch.empty((3, c.height, c.width), device=dev))
        outs.append(gstructs[si])
    r = gsr.Renderer(0)
    cfg = gsr.make_config(tile, lds, gsr.GSR_BWD_WAVE_REDUCE, thr, flags)
    torch.cuda.synchronize()
    t0 = None
    for k in range(warmup + steps):
        if k == warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        states = gsr.gsr_render_batch(r.ctx, scenes, cams, cfg, imgs)
        for im, tg, d in zip(imgs, targets, dls):
            gsr.gsr_l1_grad(r.ctx, im, tg, d)
        gsr.gsr_backward_batch(r.ctx, states, dls, outs, 0, cfg)
        for s in states:
            gsr.gsr_fwd_release(r.ctx, s)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / max(steps, 1)
    r.close()
    return {"profile_batch": spec, "views": len(mv.views), "ms_per_step": round(ms, 4)}


SERVE_RATES = (50, 100, 200, 400)       # the served stream's rates (both servers)
SERVE_RATES_HIGH = (800, 1600, 3200)    # beyond them, the batching server alone: where batches form


def _latency_stats(res):
    lat = np.array([(r.t_done - r.t_arrival) * 1000.0 for r in res])
    span = max(r.t_done for r in res) - min(r.t_arrival for r in res)
    return {"requests": len(res), "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3), "mean_ms": round(float(lat.mean()), 3),
            "steps_per_s": round(len(res) / span, 2),
            "mean_batch": round(float(np.mean([r.batch_size for r in res])), 2),
            "failed": int(sum(r.status != 0 for r in res)),
            "capacity_mode_frac": round(float(np.mean([r.render_mode == 1 for r in res])), 3),
            "reruns": int(sum(r.render_mode == 2 for r in res))}


def bench_serving(flags, seconds):
    """The served stream: ten resident scenes (100k-2M Gaussians, SH3) with Adam state on the
    device; Poisson arrivals of render + L1 + backward + Adam requests at several rates, each at
    a random eye and resolution with a device-drawn U(0,1) target. The continuous-batching server
    (wave-reduce backward, up to 16 requests per batch, two lanes), the same in capacity mode (no
    host synchronisation inside a batch), and a sequential plain-atomic server (one request at a
    time, one lane) on the same arrival streams."""
    import torch
    from paper_2401_05345_amd import gsr
    from paper_2401_05345_amd import scenegen as sg
    from paper_2401_05345_amd.serve import Server
    scenes = sg.serving_scenes()
    sizes = [s.n for s in scenes]
    log(f"[bench] serving: scenes {sizes}")
    dev = torch.device("cuda:0")
    tens = [[torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in s.arrays()] for s in scenes]
    structs = [gsr.make_scene(*t, s.sh_degree) for t, s in zip(tens, scenes)]
    resident = sum(gsr.gsr_server_scene_bytes(s.n, s.sh_degree) for s in scenes)
    # Admission at an artificial 4 GiB budget: scenes that do not fit are refused.
    admitted4 = 0
    with Server(4 << 30, max_batch=1, lanes=1) as srv:
        for st in structs:
            try:
                srv.add_scene(st)
                admitted4 += 1
            except gsr.GsrError as e:
                if e.status != gsr.GSR_EBUDGET:
                    raise
    out = {"scenes": sizes, "resident_bytes": int(resident), "admitted_at_4GiB": admitted4,
           "budget_bytes": int(resident + (8 << 30)), "rates": {}}
    reduce_cfg = gsr.make_config(16, 256, gsr.GSR_BWD_WAVE_REDUCE, 4, flags)
    plain_cfg = gsr.make_config(16, 256, gsr.GSR_BWD_PLAIN_ATOMIC, 0, flags | gsr.GSR_FLAG_ACC_F32)
    servers = {"batched_reduce": dict(max_batch=16, lanes=2, config=reduce_cfg),
               "batched_reduce_capacity": dict(max_batch=16, lanes=2, config=reduce_cfg, capacity_render=True),
               "sequential_plain": dict(max_batch=1, lanes=1, config=plain_cfg)}
    for name, kw in servers.items():
        with Server(out["budget_bytes"], lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-15, **kw) as srv:
            ids = [srv.add_scene(st) for st in structs]
            warm = sg.serving_requests(99, len(ids), 4, 100.0)
            srv.replay([srv.request(ids[si], cam, seed) for _, si, cam, seed in warm], [0.0] * len(warm))
            srv.drain()
            srv.results()
            for rate in SERVE_RATES + (SERVE_RATES_HIGH if name.startswith("batched") else ()):
                stream = sg.serving_requests(1000 + rate, len(ids), max(8, int(rate * seconds)), float(rate))
                reqs = [srv.request(ids[si], cam, seed) for _, si, cam, seed in stream]
                t0 = time.perf_counter()
                srv.replay(reqs, [t for t, _, _, _ in stream])
                srv.drain()
                res = srv.results()
                st = _latency_stats(res)
                st["wall_s"] = round(time.perf_counter() - t0, 2)
                out["rates"].setdefault(str(rate), {})[name] = st
                log(f"[bench] serve {name} {rate}/s: {st}")
    for rate, d in out["rates"].items():
        if "sequential_plain" not in d:
            continue
        d["p99_speedup"] = round(d["sequential_plain"]["p99_ms"] / d["batched_reduce"]["p99_ms"], 2)
        d["throughput_ratio"] = round(d["batched_reduce"]["steps_per_s"] / d["sequential_plain"]["steps_per_s"], 2)
    # The lowest measured rate at which requests start to share batches (mean batch >= 1.2).
    out["batches_first_form"] = {}
    for name in ("batched_reduce", "batched_reduce_capacity"):
        for rate in sorted(int(r) for r in out["rates"]):
            st = out["rates"][str(rate)].get(name)
            if st and st["mean_batch"] >= 1.2:
                out["batches_first_form"][name] = {"rate": rate, "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
                                                   "mean_batch": st["mean_batch"]}
                break
    return out


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl):
    """The fp64 oracle on the host cores, on the workload's view: its forward composite and its
    backward (composite C loop + autograd chain rule), once on one thread and once on all the
    threads this process may use (OpenMP in the per-pixel loops, torch threads in the chain
    rule). The projection and tile lists that both consume are built once, untimed."""
    import torch
    import oracle
    from oracle.composite import default_threads
    nthr = default_threads()
    out = {"kind": "oracle", "unit": "ms", "cpu_model": _cpu_model(), "host_cpus": os.cpu_count()}
    target = None
    for label, threads in (("single", 1), ("all", nthr)):
        torch.set_num_threads(threads)
        t0 = time.perf_counter()
        rr = oracle.render(wl.scene, wl.camera, threads=threads)
        t_fwd = time.perf_counter() - t0
        if target is None:
            target = oracle.render(wl.perturbed, wl.camera, threads=nthr).image if wl.perturbed is not None \
                else wl.target
            _, dl = oracle.loss_and_grad(rr.image, target, wl.loss)
        t0 = time.perf_counter()
        oracle.backward(wl.scene, rr, dl, threads=threads)
        t_bwd = time.perf_counter() - t0
        out[label] = {"threads": threads, "render_ms": round(t_fwd * 1000.0, 1),
                      "backward_ms": round(t_bwd * 1000.0, 1)}
        log(f"[bench] cpu baseline ({threads} threads): render {t_fwd:.2f} s, backward {t_bwd:.2f} s")
    out["value"] = out["all"]["backward_ms"]
    out["cores"] = nthr
    out["sample"] = (f"full backward of one {wl.camera.width}x{wl.camera.height} view of {wl.scene.n} Gaussians "
                     f"(fp64 composite backward in C + fp64 autograd chain rule) on {nthr} threads; the "
                     f"1-thread run and the fp64 forward composite (render, projection included) beside it")
    return out


def kernel_counters(kernel: str, workload: str):
    """Per-launch figures of one kernel from the committed rocprofv3 counter runs: HBM bytes
    (FETCH_SIZE and WRITE_SIZE scaled by the copy calibration) and, where taken, the VALU issue
    fraction; {} when the kernel's source changed since they were taken."""
    path = os.path.join(ROOT, "profiles", "kernel_counters.json")
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        d = json.load(f).get(kernel)
    if not d or d.get("source_hash") != source_hash(KERNEL_SOURCES[kernel]):
        return {}
    return d.get("workloads", {}).get(workload) or {}


# Sources whose text decides each measured kernel's code (the counter runs are tied to them).
KERNEL_SOURCES = {"composite_bwd": ("k_composite.hip", "device_common.hpp"),
                  "preprocess_bwd": ("k_preprocess.hip", "device_common.hpp")}


def source_hash(files=("k_composite.hip", "device_common.hpp")):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2401_05345_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def ab_legs(b, thr, iters, full=True):
    """Backward A/B on one forward state: the plain-atomic kernel with fp32 accumulators (the
    paper's baseline), the same with fp64 accumulators, and the wave-reduced kernel with both;
    with `full`, the serial-leader and block-level reductions and the plain source built with the
    compiler's own atomic reduction too. Medians in ms."""
    gsr = b.gsr
    F32 = gsr.GSR_FLAG_ACC_F32
    fr = b.forward_state(b.cfg(gsr.GSR_BWD_WAVE_REDUCE, thr))
    res = {}
    legs = [("reduce_f64", gsr.GSR_BWD_WAVE_REDUCE, thr, 0, iters),
            ("reduce_f32", gsr.GSR_BWD_WAVE_REDUCE, thr, F32, iters),
            ("plain_f32", gsr.GSR_BWD_PLAIN_ATOMIC, 0, F32, max(3, iters // 4)),
            ("plain_f64", gsr.GSR_BWD_PLAIN_ATOMIC, 0, 0, max(3, iters // 4))]
    if full:
        legs += [("serial_f64", gsr.GSR_BWD_SERIAL_REDUCE, thr, 0, iters),
                 ("block_f64", gsr.GSR_BWD_BLOCK_REDUCE, thr, 0, iters),
                 ("compiler_f64", gsr.GSR_BWD_PLAIN_COMPILER_REDUCE, 0, 0, max(3, iters // 4)),
                 ("compiler_f32", gsr.GSR_BWD_PLAIN_COMPILER_REDUCE, 0, F32, max(3, iters // 4))]
    for name, mode, t, flags, n in legs:
        z = []
        a6, a7 = b.backward_only(fr, b.cfg(mode, t, flags), n, z)
        res[name] = (float(np.median(a6)), float(np.median(a7)), float(np.median(z)))
    cnt = {"plain": b.counters(fr, gsr.GSR_BWD_PLAIN_ATOMIC, 0), "reduce": b.counters(fr, gsr.GSR_BWD_WAVE_REDUCE, thr)}
    if full:
        cnt["block"] = b.counters(fr, gsr.GSR_BWD_BLOCK_REDUCE, thr)
    stats = fr.stats
    b.r.release(fr)
    return res, cnt, stats


def ab_summary(res, cnt, stats, thr, sweep):
    r6, r7, rz = res["reduce_f64"]
    p6, p7, pz = res["plain_f32"]
    q6, q7, qz = res["plain_f64"]
    w6, w7, wz = res["reduce_f32"]
    cp, cr = cnt["plain"], cnt["reduce"]
    out = {
        "n_pairs": int(stats.n_pairs), "n_visible": int(stats.n_visible), "threshold": thr,
        "wave_reduce_ms": round(rz + r6 + r7, 4),
        "plain_atomic_ms": round(pz + p6 + p7, 4),
        "plain_atomic_f64_ms": round(qz + q6 + q7, 4),
        "wave_reduce_acc_f32_ms": round(wz + w6 + w7, 4),
        "clear_and_tile_order_ms": round(rz, 4),
        "composite_bwd_wave_reduce_ms": round(r6, 4),
        "preprocess_bwd_ms": round(r7, 4),
        "composite_bwd_plain_ms": round(p6, 4),
        "speedup_composite_bwd": round(p6 / r6, 3),
        "speedup_composite_bwd_both_f32": round(p6 / w6, 3),
        "speedup_composite_bwd_both_f64": round(q6 / r6, 3),
        "lane_atomics_plain": int(cp.lane_atomics), "lane_atomics_reduce": int(cr.lane_atomics),
        "atomic_instrs_plain": int(cp.atomic_instrs), "atomic_instrs_reduce": int(cr.atomic_instrs),
        "evaluated_E": int(cr.evaluated), "active_A": int(cr.active), "wave_entries": int(cr.wave_entries),
        "visited_wave_entries": int(cr.visited), "longest_wave_walk": int(cr.max_wave_visits),
        "walked_entries_P_walk": int(cr.walked),
        "reduced_W_R": int(cr.reduced), "plain_lanes_A_lt": int(cr.plain_lanes),
        "threshold_sweep_ms": sweep,
        "accumulator_note": ("fp64 accumulators (default) meet the 1e-3 gradient tolerance against the oracle; "
                             "fp32 accumulators (the paper's setting, both *_acc_f32 / plain_atomic legs) add "
                             "each value in an order the atomics decide, and on views with screen-filling "
                             "splats (3M/1080p) their run-to-run spread exceeds 1e-3: outside parity there"),
    }
    if "serial_f64" in res:
        out["composite_bwd_by_mode_ms"] = {
            "f64_accumulators": {"wave_reduce": round(r6, 4), "serial_leader": round(res["serial_f64"][0], 4),
                                 "block_lds": round(res["block_f64"][0], 4), "plain_atomic": round(q6, 4),
                                 "plain_compiler_reduced": round(res["compiler_f64"][0], 4)},
            "f32_accumulators": {"wave_reduce": round(w6, 4), "plain_atomic": round(p6, 4),
                                 "plain_compiler_reduced": round(res["compiler_f32"][0], 4)}}
        out["speedup_composite_bwd_vs_compiler_reduced"] = round(res["compiler_f64"][0] / r6, 3)
        out["lane_atomics_block_lds"] = int(cnt["block"].lane_atomics)
        out["atomic_instrs_block_lds"] = int(cnt["block"].atomic_instrs)
    return out


def rooflines(wl, stats, cr, a6_ms, a7_ms):
    """Both backward kernels against their roofs, from the live event timings: the composite
    (a6) against the fp32 vector peak, the per-Gaussian chain rule (a7) against HBM."""
    hw = wl.camera.width * wl.camera.height
    n, n_vis = wl.scene.n, int(stats.n_visible)
    K3 = 3 * (wl.scene.sh_degree + 1) ** 2
    flops = FLOPS_PER_EVAL * cr.evaluated + FLOPS_PER_CONTRIB * cr.active + FLOPS_PER_REDUCED * cr.reduced
    a6_tflops = flops / (a6_ms * 1e-3) / 1e12
    pbytes = 4 * (11 + K3)
    # records: the entries the blocks stage (P_walk: each tile's block walks to its deepest pixel's
    # n_contrib), not all P entries of the lists
    a6_bytes = BYTES_PER_PIXEL * hw + BYTES_PER_VISIBLE * n_vis + BYTES_PER_RECORD * int(cr.walked)
    a6 = {"bound": "alu", "achieved": round(a6_tflops, 3), "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
          "frac": round(a6_tflops / PEAK_FP32_VALU_TFLOPS, 4), "kernel": "composite_bwd_kernel<16,256,wave_reduce>",
          "ms": round(a6_ms, 4), "algorithmic_flops": int(flops), "algorithmic_bytes": int(a6_bytes),
          "hbm_GBs_algorithmic": round(a6_bytes / (a6_ms * 1e-3) / 1e9, 1),
          "hbm_frac_algorithmic": round(a6_bytes / (a6_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
    m6 = kernel_counters("composite_bwd", wl.name)
    a6["traffic"] = m6.get("bytes_per_launch")
    if "valu_issue_frac" in m6:
        a6["valu_issue_frac"] = m6["valu_issue_frac"]
    # a7: reads radius (4 B) of every Gaussian and, for the visible ones, the parameters and the nine
    # fp64 accumulator sums; writes every Gaussian's gradient row (zeros for culled ones).
    a7_bytes = n * (4 + pbytes) + n_vis * (pbytes + 72)
    a7_gbs = a7_bytes / (a7_ms * 1e-3) / 1e9
    a7 = {"bound": "hbm", "achieved": round(a7_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
          "frac": round(a7_gbs / PEAK_HBM_GBS, 4), "kernel": f"preprocess_bwd_kernel<{wl.scene.sh_degree},double>",
          "ms": round(a7_ms, 4), "algorithmic_bytes": int(a7_bytes)}
    m7 = kernel_counters("preprocess_bwd", wl.name)
    a7["traffic"] = m7.get("bytes_per_launch")
    dom, other = (a7, a6) if a7_ms >= a6_ms else (a6, a7)
    line = dict(dom)
    line["other_backward_kernel"] = other
    return line


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU sharding of this "
              f"path is a design note, not a measured configuration.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2401_05345_amd import gsr
    from paper_2401_05345_amd import scenegen as sg
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n * 4, "launches": 5}))
        return
    gsr.load()
    if args.microbench:
        kind, mib = args.microbench.split(":")
        kinds = {"write": gsr.GSR_MB_WRITE, "read": gsr.GSR_MB_READ, "copy_nt": gsr.GSR_MB_COPY_NT,
                 "gather48": gsr.GSR_MB_GATHER48, "copy": gsr.GSR_MB_COPY}
        r = gsr.Renderer(0)
        ms, ops = gsr.gsr_microbench(r.ctx, kinds[kind], int(mib) << 20, reps=5)
        r.close()
        print(json.dumps({"microbench": kind, "bytes": int(mib) << 20, "bytes_per_launch": ops, "ms": ms,
                          "GBs": round(ops / ms / 1e6, 1), "launches": 6}))
        return

    if args.serve_only:
        flags = 0 if args.no_lane_split else gsr.GSR_FLAG_LANE_SPLIT_ATOMICS
        print(json.dumps({"serving": bench_serving(flags, args.serve_seconds)}))
        return

    if args.profile_batch:
        flags = 0 if args.no_lane_split else gsr.GSR_FLAG_LANE_SPLIT_ATOMICS
        print(json.dumps(profile_multi_view(flags, args.profile_batch, args.steps, args.warmup)))
        return

    wl = sg.WORKLOADS[args.workload]()
    log(f"[bench] workload {wl.name}: {wl.scene.n} Gaussians, {wl.camera.width}x{wl.camera.height}")
    Bench.extra_flags = ((0 if args.no_lane_split else gsr.GSR_FLAG_LANE_SPLIT_ATOMICS) |
                         (gsr.GSR_FLAG_XCD_REMAP if args.xcd_remap else 0) |
                         (gsr.GSR_FLAG_NO_TILE_ORDER if args.no_tile_order else 0))
    b = Bench(wl)

    # Threshold: one backward per candidate on a warm forward state (the paper's tuning rule).
    sweep = None
    if args.threshold is None and not args.profile_only:
        fr = b.forward_state(b.cfg(gsr.GSR_BWD_WAVE_REDUCE, 32))
        b.backward_only(fr, b.cfg(gsr.GSR_BWD_WAVE_REDUCE, 32), 2)
        sweep = b.sweep(fr)
        thr = min(sweep, key=sweep.get)
        log(f"[bench] threshold sweep (a6 ms): {sweep} -> {thr}")
        b.r.release(fr)
    else:
        # Profiled runs launch only the configuration they measure.
        thr = args.threshold if args.threshold is not None else 32

    cfg_r = b.cfg(MODES[args.mode], thr)
    for _ in range(args.warmup):
        b.step(cfg_r)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per = []
    stats = None
    for _ in range(args.steps):
        st, stats = b.step(cfg_r)
        per.append(st)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1000.0 / args.steps
    # The whole backward call: accumulator rows cleared, backward composite, per-Gaussian chain rule.
    bwd = np.array([s.zero_acc + s.composite_bwd + s.preprocess_bwd for s in per])
    a6 = np.array([s.composite_bwd for s in per])
    fwd = np.array([s.preprocess + s.depth_sort + s.scan_emit + s.tile_sort + s.ranges + s.composite_fwd for s in per])
    a7 = np.array([s.preprocess_bwd for s in per])
    log(f"[bench] {args.steps} steps: {wall:.3f} ms/step, backward {bwd.mean():.3f} ms (a6 {a6.mean():.3f}, "
        f"a7 {a7.mean():.3f})")
    stages = {k: round(float(np.mean([getattr(s, k) for s in per])), 4)
              for k in ("preprocess", "depth_sort", "scan_emit", "tile_sort", "ranges", "composite_fwd")}
    log(f"[bench] render {fwd.mean():.4f} ms, stages {stages}")
    if args.profile_only:
        print(json.dumps({"profile_only": True, "ms_per_step": wall, "bwd_ms": float(bwd.mean()),
                          "render_ms": float(fwd.mean()), "forward_stages_ms": stages}))
        return

    # A/B on one forward state: plain atomics vs wave reduce, same inputs.
    res, cnt, fstats = ab_legs(b, thr, max(10, args.steps))
    backward = ab_summary(res, cnt, fstats, thr, sweep)
    backward["p50_backward_ms"] = round(float(np.percentile(bwd, 50)), 4)
    backward["p99_backward_ms"] = round(float(np.percentile(bwd, 99)), 4)
    log(f"[bench] A/B a6: plain {res['plain_f32'][0]:.3f} ms, reduce {res['reduce_f64'][0]:.3f} ms")
    # The kernels' launch times over the timed region (its steps' events), when it runs the
    # wave-reduced backward; the A/B legs repeat the backward on one warm state and run a few
    # per cent faster.
    if MODES[args.mode] == gsr.GSR_BWD_WAVE_REDUCE:
        roofline = rooflines(wl, fstats, cnt["reduce"], float(a6.mean()), float(a7.mean()))
        roofline["timing"] = f"mean over the {args.steps} timed steps"
    else:
        roofline = rooflines(wl, fstats, cnt["reduce"], res["reduce_f64"][0], res["reduce_f64"][1])
        roofline["timing"] = "median of the wave-reduce A/B leg"

    out = {
        "metric": "3DGS backward ms/iter + TCC atomics, wave-reduce vs plain atomics; p99 step lat",
        "value": round(float(bwd.mean()), 4),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "n_gaussians": wl.scene.n, "width": wl.camera.width,
                   "height": wl.camera.height, "sh_degree": wl.scene.sh_degree, "tile": 16, "lds_batch": 256,
                   "bwd_mode": "wave_reduce", "reduce_threshold": thr, "accumulators": "f64",
                   "loss": wl.loss, "n_pairs": int(stats.n_pairs), "n_visible": int(stats.n_visible)},
        "roofline": roofline,
        "backward": backward,
        "forward_ms": round(float(fwd.mean()), 4),
        "forward_stages_ms": stages,
        "p99_step_ms": None,
    }

    # Measured roofs (micro-benchmarks of the kernels' memory patterns) and a6 against them.
    try:
        roofs = measure_roofs(b.r.ctx)
        out["roofs"] = roofs
        cp, cr = cnt["plain"], cnt["reduce"]
        plain_rate = cp.lane_atomics / (res["plain_f32"][0] * 1e-3)
        red_rate = cr.lane_atomics / (res["reduce_f64"][0] * 1e-3)
        out["backward"]["atomic_roofline"] = {
            "plain": {"pattern": "f32_same_address_16MiB", "achieved_lane_ops_s": round(plain_rate / 1e9, 3),
                      "peak_lane_ops_s": roofs["atomic_Gops"]["f32_same_address_16MiB"],
                      "frac": round(plain_rate / 1e9 / roofs["atomic_Gops"]["f32_same_address_16MiB"], 4),
                      "unit": "G lane-ops/s"},
            "wave_reduce": {"pattern": "f64_nine_lanes_16MiB", "achieved_lane_ops_s": round(red_rate / 1e9, 3),
                            "peak_lane_ops_s": roofs["atomic_Gops"]["f64_nine_lanes_16MiB"],
                            "frac": round(red_rate / 1e9 / roofs["atomic_Gops"]["f64_nine_lanes_16MiB"], 4),
                            "unit": "G lane-ops/s"}}
        if roofline["unit"] == "GB/s":
            roofline["frac_of_measured_write_roof"] = round(roofline["achieved"] / roofs["hbm_write_GBs"], 4)
    except Exception as e:  # noqa: BLE001
        log(f"[bench] roof micro-benchmarks failed: {e!r}")
        out["roofs"] = {"error": repr(e)}
    b.r.close()

    # The object-centred 100k-Gaussian 800x800 view: the same A/B as an extra leg.
    if not args.no_object and args.workload != "object_100k":
        wl2 = sg.object_100k()
        log(f"[bench] A/B at {wl2.name}")
        b2 = Bench(wl2)
        fr2 = b2.forward_state(b2.cfg(gsr.GSR_BWD_WAVE_REDUCE, 32))
        s2 = b2.sweep(fr2, iters=2)
        thr2 = min(s2, key=s2.get)
        b2.r.release(fr2)
        per2 = []
        for k in range(13):
            st2, _ = b2.step(b2.cfg(gsr.GSR_BWD_WAVE_REDUCE, thr2))
            if k >= 3:
                per2.append(st2)
        res2, cnt2, stats2 = ab_legs(b2, thr2, 10)
        leg = ab_summary(res2, cnt2, stats2, thr2, s2)
        leg["roofline"] = rooflines(wl2, stats2, cnt2["reduce"], float(np.mean([s.composite_bwd for s in per2])),
                                    float(np.mean([s.preprocess_bwd for s in per2])))
        leg["roofline"]["timing"] = f"mean over {len(per2)} steps"
        leg["step_render_ms"] = round(float(np.mean([s.preprocess + s.depth_sort + s.scan_emit + s.tile_sort +
                                                     s.ranges + s.composite_fwd for s in per2])), 4)
        leg["forward_stages_ms"] = {k: round(float(np.mean([getattr(s, k) for s in per2])), 4)
                                    for k in ("preprocess", "depth_sort", "scan_emit", "tile_sort", "ranges",
                                              "composite_fwd")}
        out[wl2.name] = leg
        b2.r.close()

    # The extra legs report their own failure instead of losing the line.
    if not args.no_batch:
        try:
            out["multi_view_16"] = bench_multi_view(Bench.extra_flags)
        except Exception as e:  # noqa: BLE001
            log(f"[bench] multi-view leg failed: {e!r}")
            out["multi_view_16"] = {"error": repr(e)}

    if not args.no_serve:
        try:
            out["serving"] = bench_serving(Bench.extra_flags, args.serve_seconds)
            out["p99_step_ms"] = out["serving"]["rates"]["200"]["batched_reduce"]["p99_ms"]
        except Exception as e:  # noqa: BLE001
            log(f"[bench] serving leg failed: {e!r}")
            out["serving"] = {"error": repr(e)}

    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
