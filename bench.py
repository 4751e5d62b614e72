#!/usr/bin/env python3
"""Throughput of plain FSR/SSR spike-stream reconstruction on one MI355X.

Workload: 250x400 pixels, 20000 frames (1 s at 20 kHz) of moving gratings
plus a rotating sectored disk with Poisson photon noise (seed 2), intensity
reconstructed at every 10th frame (2000 output planes).  One step = one
spk_reconstruct call over the whole stream (ingest, transpose, spike
intervals, FSR + SSR segmentation, Eq. 6 intensity, output writes), with the
packed stream already resident in HBM.

Prints one JSON line.  Also:
  --parse-rocprof DIR   summarise rocprofv3 output (kernel stats or PMC
                        counters) found under DIR as text, for profiles/.
"""
from __future__ import annotations

import argparse
import ctypes
import csv
import glob
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "recon Mpixel-frames/s + %HBM peak; surrogate vs plain at ≥40 dB PSNR"
HBM_PEAK_GBS = 8000.0
KERNEL_NAME = "recon_kernel"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_recon_gratings_250x400_T20000.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2412_11639_amd", "csrc", f)
                  for f in ("recon.hip", "recon_core.h", "spk_internal.h")]


def kernel_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(H, W, T, n_out) -> int:
    """One bit in per pixel-frame, one float32 out per pixel per output."""
    return T * H * W // 8 + n_out * H * W * 4


def load_counters(order_name):
    """Counter figures per step (HBM bytes, VALU instructions) from the
    committed summary, if it was taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return {}
    if t.get("kernel_sha") != kernel_sha():
        return {}
    return t.get("per_order", {}).get(order_name, {})


# integer VALU issue: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD every
# 4 cycles (16 lanes wide), 2.4 GHz
VALU_PEAK_PER_S = 256 * 2.4e9


COPY_BYTES = 1 << 30  # the calibration copy moves 1 GiB each way


def _counter_means(d: str):
    """(kernel name, counter) -> mean value per dispatch, from rocprofv3
    output under d (rocpd SQLite databases or counter_collection CSVs)."""
    import sqlite3
    acc = {}
    for f in glob.glob(os.path.join(d, "**", "*_results.db"), recursive=True):
        con = sqlite3.connect(f)
        try:
            for name, cname, v in con.execute(
                    "select kernel_name, counter_name, value from counters_collection"):
                acc.setdefault((name, cname), []).append(v)
        except sqlite3.Error:
            pass
        con.close()
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                acc.setdefault((r["Kernel_Name"], r["Counter_Name"]), []).append(
                    float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def traffic_from_counters(d: str):
    """HBM bytes per reconstruction step (recon_kernel + fixup_kernel) of each
    order from the FETCH_SIZE and WRITE_SIZE passes under d, each scaled by
    what the same counter reads for the 1 GiB calibration copy in the same
    run."""
    vals = _counter_means(d)
    out = {}
    for cname in ("FETCH_SIZE", "WRITE_SIZE"):
        copy = [v for (n, c), v in vals.items() if c == cname and "copyBuffer" in n]
        if not copy:
            continue
        factor = COPY_BYTES / (copy[0] * 1024.0)
        for (n, c), v in vals.items():
            if c != cname:
                continue
            for kern in ("recon_kernel", "fixup_kernel"):
                for o, key in (("1", "FSR"), ("2", "SSR")):
                    if kern + "<" + o + ", 0, false, 0>" in n:
                        e = out.setdefault(key, {}).setdefault(cname, {"factor": factor})
                        e[kern + "_kib"] = v
                        e["bytes"] = e.get("bytes", 0.0) + v * 1024.0 * factor
    # VALU instructions (wave64) per step, when an SQ pass is present
    for (n, c), v in vals.items():
        if c != "SQ_INSTS_VALU":
            continue
        for kern in ("recon_kernel", "fixup_kernel"):
            for o, key in (("1", "FSR"), ("2", "SSR")):
                if kern + "<" + o + ", 0, false, 0>" in n:
                    e = out.setdefault(key, {})
                    e["valu_per_launch"] = e.get("valu_per_launch", 0.0) + v
    for key, d2 in out.items():
        if "FETCH_SIZE" in d2 and "WRITE_SIZE" in d2:
            d2["hbm_bytes_per_launch"] = d2["FETCH_SIZE"]["bytes"] + d2["WRITE_SIZE"]["bytes"]
    return out


def run_small(spk, spkgen, torch, np):
    """The small static configuration: 250x400 blocks, 1024 frames, 8
    outputs at 64 + 128 k.  16 MB of algorithmic bytes per call, so a call
    is bound by launch and latency, not HBM: timed as the mean of 200 calls
    (HIP events around the loop) for SSR and FSR."""
    wl = spkgen.BLOCKS_250x400
    H, W, T = wl.H, wl.W, wl.T
    t_out = wl.times().tolist()
    ds = torch.from_numpy(wl.generate()).cuda()
    out = torch.empty((len(t_out), H, W), dtype=torch.float32, device="cuda")
    res = {"workload": wl.name, "n_out": len(t_out),
           "algorithmic_bytes": algorithmic_bytes(H, W, T, len(t_out))}
    for name, order in (("SSR", spk.SSR), ("FSR", spk.FSR)):
        for _ in range(10):
            spk.reconstruct(ds, H, W, T, 1.0, t_out, order=order, out=out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(200):
            spk.reconstruct(ds, H, W, T, 1.0, t_out, order=order, out=out)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 200
        gbs = res["algorithmic_bytes"] / (ms * 1e-3) / 1e9
        res[name] = {"ms": round(ms, 4), "mpx_frames_per_s": round(H * W * T / (ms * 1e-3) / 1e6, 1),
                     "achieved_GBs": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
    del ds, out
    return res


def run_batched(args, spk, spkgen, torch, np):
    """16 streams of uneven size, 4096 frames each, 64 outputs each, in one
    autotuned plan (persistent kernel in a HIP graph).  Returns the result
    and the smallest stream with its GPU output, for the CPU leg."""
    jobs = spkgen.batch_workload()
    order = spk.SSR if args.order == "ssr" else spk.FSR
    print("batched: generating %d streams" % len(jobs), file=sys.stderr, flush=True)
    dev_jobs, host0 = [], None
    for j in jobs:
        s = spkgen.blocks(j["H"], j["W"], j["T"], j["seed"])
        if host0 is None or j["H"] * j["W"] < host0[1]["H"] * host0[1]["W"]:
            host0 = (s, j, len(dev_jobs))
        dev_jobs.append(dict(j, stream=torch.from_numpy(s).cuda()))
        del s
    plan = spk.Plan(dev_jobs, order=order, autotune=True)
    for _ in range(args.warmup):
        plan.execute()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        plan.execute()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    px_frames = sum(j["H"] * j["W"] * j["T"] for j in jobs)
    alg = sum(algorithmic_bytes(j["H"], j["W"], j["T"], len(j["t_out"])) for j in jobs)
    s0, j0, idx = host0
    check = dict(stream=s0, job=j0, order=order, got=plan.outputs()[idx].cpu().numpy())
    info = dict(plan.info(), **plan.shape())
    plan.close()
    del dev_jobs
    torch.cuda.empty_cache()
    return {"workload": "batch16_mixed_T4096_64out", "order": args.order.upper(),
            "streams": len(jobs), "pixels": sum(j["H"] * j["W"] for j in jobs),
            "ms_per_step": round(ms, 4), "value": round(px_frames / (ms * 1e-3) / 1e6, 1),
            "unit": "Mpixel-frames/s", "achieved_GBs": round(alg / (ms * 1e-3) / 1e9, 1),
            "frac_hbm": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "launch": info, "graph": True, "autotuned": True}, check


SUR_FLOP_PER_PX = 2 * 28224       # forward multiply-adds of the 4 conv layers
# training: forward + input gradients of layers 2-4 + weight gradients of all 4
SUR_TRAIN_FLOP_PER_PX = 3 * SUR_FLOP_PER_PX - 2 * 9 * 33 * 32
MFMA_BF16_PEAK_TFLOPS = 2500.0


def _psnr(x, ref, np):
    """10 log10(theta^2 / MSE) with theta = 1."""
    mse = float(np.mean((np.asarray(x, np.float64) - np.asarray(ref, np.float64)) ** 2))
    return 10.0 * np.log10(1.0 / mse) if mse > 0 else float("inf")


def run_surrogate(args, spk, spkgen, torch, np):
    """Surrogate training on seeded static block scenes (250x400x4096;
    targets = the plain method over the whole stream, computed by the
    library), held-out outputs, and the 1000x1000 streaming run."""
    import paper_2412_11639_amd.surrogate as sur
    out, checks = {}, {}
    H, W, T = 250, 400, 4096
    t0 = time.perf_counter()
    print("surrogate: %d training scenes" % args.sur_scenes, file=sys.stderr, flush=True)
    scenes = sur.SceneSet([10000 + i for i in range(args.sur_scenes)], H=H, W=W, T=T)
    held = sur.SceneSet([20000 + i for i in range(32)], H=H, W=W, T=T)
    gen_s = time.perf_counter() - t0
    B, Hc, Wc, lr = 32, 64, 64, 3e-4
    # warm-up: a few eager steps (kernels loaded, launch caches filled)
    sur.train(sur.Surrogate(seed=0), scenes, steps=20, B=B, Hc=Hc, Wc=Wc, lr=lr, seed=99)
    # the timed run: the same crops and learning rates as sur.train(seed=1),
    # every step replayed from the captured graph of a training plan
    model = sur.Surrogate(seed=0)
    rng = np.random.default_rng(1)
    steps = args.sur_steps
    plan = sur.TrainPlan(model, [scenes.samples(rng, B, Hc, Wc) for _ in range(steps)],
                         [lr * 0.5 * (1 + math.cos(math.pi * k / steps)) for k in range(steps)],
                         Hc, Wc)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    print("surrogate: training %d steps" % steps, file=sys.stderr, flush=True)
    e0.record()
    plan.run(steps)
    e1.record()
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / steps
    per = plan.losses()
    plan.close()
    chunk = max(1, steps // 6)
    losses = [float(per[k:k + chunk].mean()) for k in range(0, steps, chunk)]
    # held-out outputs at two times per scene, whole frames
    eval_times = [held.target_times[1], held.target_times[3]]
    ys, ests, muxs, plain_long = [], [], [], []
    for i in range(len(held.seeds)):
        for k, t in enumerate(eval_times):
            smp = [dict(stream=held.streams[i], H=H, W=W, T=T, oy=0, ox=0, t=t)]
            win, est, st = sur.Surrogate.input(smp, H, W, 1.0)
            y = model.forward(win, est)
            ys.append(y[0].cpu().numpy())
            ests.append(est[0].cpu().numpy())
            muxs.append(sur.Surrogate.mux(y, est, st)[0].cpu().numpy())
            plain_long.append(held.targets[i][held.target_times.index(t)].cpu().numpy())
    train_tflops = SUR_TRAIN_FLOP_PER_PX * B * Hc * Wc / (ms_step * 1e-3) / 1e12
    out["surrogate"] = {
        "workload": "blocks_250x400_T4096: %d training scenes (seeds 10000+), 32 held out "
                    "(seeds 20000-20031), outputs at t=%s" % (args.sur_scenes, eval_times),
        "train_steps": args.sur_steps, "batch": "%d crops of %dx%d" % (B, Hc, Wc), "lr": lr,
        "train_ms_per_step": round(ms_step, 3), "train_tflops": round(train_tflops, 2),
        "train_mfma_frac": round(train_tflops / MFMA_BF16_PEAK_TFLOPS, 5),
        "loss_curve": [float("%.4g" % l) for l in losses], "data_gen_s": round(gen_s, 1)}
    checks["surrogate"] = dict(host=held.host, H=H, W=W, T=T, times=eval_times,
                               y=np.stack(ys), est=np.stack(ests), mux=np.stack(muxs),
                               plain_long=np.stack(plain_long))
    # the same training step at the largest batch the plans take (64 crops
    # of 128x128, 1 M px per step): the step's MFMA utilisation when
    # launch latency is amortised (timing only; the network is discarded)
    Bl, Hl, Wl, nl = 64, 128, 128, 60
    big = sur.Surrogate(seed=0)
    rng_l = np.random.default_rng(3)
    plan = sur.TrainPlan(big, [scenes.samples(rng_l, Bl, Hl, Wl) for _ in range(nl)],
                         [lr] * nl, Hl, Wl)
    plan.run(10)
    torch.cuda.synchronize()
    e0.record()
    plan.run(nl - 10)
    e1.record()
    torch.cuda.synchronize()
    ms_l = e0.elapsed_time(e1) / (nl - 10)
    plan.close()
    del big
    tf_l = SUR_TRAIN_FLOP_PER_PX * Bl * Hl * Wl / (ms_l * 1e-3) / 1e12
    out["surrogate"]["large_batch_step"] = {
        "batch": "%d crops of %dx%d" % (Bl, Hl, Wl), "ms_per_step": round(ms_l, 4),
        "tflops": round(tf_l, 2), "mfma_frac": round(tf_l / MFMA_BF16_PEAK_TFLOPS, 5)}
    del scenes, held
    torch.cuda.empty_cache()
    # a second network for the moving streaming scene: the same training on
    # block scenes that translate at up to 2 px/frame (the streaming
    # scene's generator, other seeds), whole-stream targets
    t0 = time.perf_counter()
    print("surrogate: %d moving training scenes" % args.sur_moving_scenes, file=sys.stderr,
          flush=True)
    mscenes = sur.SceneSet([40000 + i for i in range(args.sur_moving_scenes)], H=H, W=W, T=T,
                           moving=True, keep_host=False)
    mgen_s = time.perf_counter() - t0
    motion = sur.Surrogate(seed=0)
    rng = np.random.default_rng(2)
    plan = sur.TrainPlan(motion, [mscenes.samples(rng, B, Hc, Wc) for _ in range(steps)],
                         [lr * 0.5 * (1 + math.cos(math.pi * k / steps)) for k in range(steps)],
                         Hc, Wc)
    e0.record()
    plan.run(steps)
    e1.record()
    torch.cuda.synchronize()
    mper = plan.losses()
    out["surrogate"]["moving_model"] = {
        "workload": "blocks_250x400_T4096 translating at up to 2 px/frame: %d training scenes "
                    "(seeds 40000+), whole-stream targets" % args.sur_moving_scenes,
        "train_steps": steps, "train_ms_per_step": round(e0.elapsed_time(e1) / steps, 3),
        "loss_curve": [float("%.4g" % float(mper[k:k + chunk].mean()))
                       for k in range(0, steps, chunk)],
        "data_gen_s": round(mgen_s, 1)}
    plan.close()
    del mscenes
    torch.cuda.empty_cache()
    out["streaming"], checks["streaming"] = run_streaming(args, spk, spkgen, torch, np, motion,
                                                          sur, static_model=model)
    return out, checks


def _streaming_scene(spkgen, np, H, W, T):
    """The streaming workload: blocks translating at one velocity,
    |v| in (0, 2] px/frame, direction and speed from seed 5."""
    import paper_2412_11639_amd.surrogate as sur
    vx, vy = sur.scene_velocity(5)
    speed = math.hypot(vx, vy)
    print("streaming: generating %dx%dx%d" % (H, W, T), file=sys.stderr, flush=True)
    return spkgen.blocks(H, W, T, 5, vx=vx, vy=vy), speed, vx, vy


def _encoded_leg(spk, torch, ds, H, W, T, frames, out, ref_idx, ref_kept, packed=True):
    """The plain method through the segment encoding (FSR): spk_segments
    writes each pixel's segment list, spk_decode expands it to every frame
    in ``frames`` (into ``out``); with ``packed`` the lists are laid out per
    pixel (spk_segments_packed / spk_decode_packed), else as [cap][H*W]
    arrays.  Times both on the second of two runs; ``ref_kept`` (planes
    ``ref_idx`` of the single-pass output) checks the decoded frames.  The
    decoder's roofline is HBM: algorithmic bytes are the lists it reads
    (12 B per segment plus the counts) and the frames it writes."""
    cnt = spk.segments(ds, H, W, T, order=spk.FSR, cap=0)[3]
    cap = max(1, int(cnt.max().item()))
    if packed:
        seg = [torch.empty((H * W, cap, 3), dtype=torch.int32, device="cuda")]
    else:
        seg = [torch.empty((cap, H * W), dtype=torch.int32, device="cuda") for _ in range(3)]
    lib = spk._lib.load()
    tp = (ctypes.c_int32 * len(frames))(*frames)
    e0, e_mid, e1 = (torch.cuda.Event(enable_timing=True) for _ in range(3))

    def encoded():
        st = torch.cuda.current_stream().cuda_stream
        if packed:
            rc = lib.spk_segments_packed(ds.data_ptr(), H, W, T, spk.FSR, cap, seg[0].data_ptr(),
                                         cnt.data_ptr(), st)
            e_mid.record()
            rc |= lib.spk_decode_packed(seg[0].data_ptr(), cnt.data_ptr(), cap, H, W, T, 1.0, tp,
                                        len(frames), out.data_ptr(), st)
        else:
            rc = lib.spk_segments(ds.data_ptr(), H, W, T, spk.FSR, cap, seg[0].data_ptr(),
                                  seg[1].data_ptr(), seg[2].data_ptr(), cnt.data_ptr(), st)
            e_mid.record()
            rc |= lib.spk_decode(seg[0].data_ptr(), seg[1].data_ptr(), seg[2].data_ptr(),
                                 cnt.data_ptr(), cap, H, W, T, 1.0, tp, len(frames),
                                 out.data_ptr(), st)
        assert rc == 0

    encoded()
    torch.cuda.synchronize()
    e0.record()
    encoded()
    e1.record()
    torch.cuda.synchronize()
    enc_ms, dec_ms = e0.elapsed_time(e_mid), e_mid.elapsed_time(e1)
    same = bool(torch.equal(out[ref_idx].cpu(), torch.from_numpy(ref_kept)))
    seg_bytes = int(cnt.sum().item()) * 12
    dec_bytes = seg_bytes + H * W * 4 + len(frames) * H * W * 4
    achieved = dec_bytes / (dec_ms * 1e-3) / 1e9
    del seg
    torch.cuda.empty_cache()
    return {"layout": "per pixel [H*W][cap][3]" if packed else "[cap][H*W] x 3",
            "mpx_frames_per_s": round(H * W * T / ((enc_ms + dec_ms) * 1e-3) / 1e6, 1),
            "segments_ms": round(enc_ms, 3), "decode_ms": round(dec_ms, 3),
            "segment_bytes": seg_bytes, "cap": cap, "equals_single_pass": same,
            "decode_roofline": {"bound": "hbm", "achieved": round(achieved, 1),
                                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": round(achieved / HBM_PEAK_GBS, 4),
                                "algorithmic_bytes": dec_bytes}}


def other_paths(spk, torch, ds, H, W, T, t_out, out):
    """The other per-pixel paths on the bench stream with the same 2000
    outputs: the third order and TFI through the reconstruction kernel, the
    TFP-32 baseline and the static/motion mask (SSR, 64-frame window).
    Each: time per call (2 warm-up, 5 timed, HIP events) and its
    algorithmic bytes against the 8 TB/s HBM peak."""
    n_out, HW = len(t_out), H * W
    rec = algorithmic_bytes(H, W, T, n_out)
    legs = {
        "third_order": (lambda: spk.reconstruct(ds, H, W, T, 1.0, t_out, order=spk.TSR, out=out),
                        rec, "T/8 B in + 4 B per pixel-output"),
        "TFI": (lambda: spk.reconstruct(ds, H, W, T, 1.0, t_out, order=spk.TFI, out=out),
                rec, "T/8 B in + 4 B per pixel-output"),
        "TFP-32": (lambda: spk.tfp(ds, H, W, T, 1.0, 32, t_out, out=out),
                   n_out * HW * (32 // 8 + 4), "32/8 B in + 4 B out per pixel-output"),
        "motion_SSR_64": (lambda: spk.motion(ds, H, W, T, 64, t_out, order=spk.SSR),
                          T * HW // 8 + n_out * HW, "T/8 B in + 1 B per pixel-output"),
    }
    res = {}
    for name, (fn, nbytes, what) in legs.items():
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        gbs = nbytes / (ms * 1e-3) / 1e9
        res[name] = {"ms": round(ms, 4),
                     "mpx_frames_per_s": round(HW * T / (ms * 1e-3) / 1e6, 1),
                     "algorithmic_bytes": nbytes, "bytes": what,
                     "achieved_GBs": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
    return res


def run_forward(args, spk, spkgen, torch, np):
    """The surrogate forward alone at 1000x1000: the window and estimate of
    the streaming scene after 64 frames, 50 timed inferences (random-init
    weights, seed 0: the cost does not depend on them)."""
    import paper_2412_11639_amd.surrogate as sur
    H = W = 1000
    s, _, _, _ = _streaming_scene(spkgen, np, H, W, 64)
    ds = torch.from_numpy(s).cuda()
    win = torch.zeros((1, H, W), dtype=torch.int32, device="cuda")
    est = torch.zeros((1, H, W), dtype=torch.float32, device="cuda")
    st = torch.zeros((1, H, W), dtype=torch.uint8, device="cuda")
    for t in range(64):
        sur.Surrogate.stream_step(ds[t], H, W, 1.0, win, est, st)
    model = sur.Surrogate(seed=0)
    y = torch.empty((1, H, W), dtype=torch.float32, device="cuda")
    for _ in range(5):
        model.infer(win, est, out=y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(50):
        model.infer(win, est, out=y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 50
    return {"workload": "surrogate forward 1000x1000 (window and estimate of the streaming "
                        "scene after 64 frames)",
            "ms": round(ms, 4),
            "mfma_frac": round(SUR_FLOP_PER_PX * H * W / (ms * 1e-3) / 1e12 / MFMA_BF16_PEAK_TFLOPS,
                               4),
            "algorithmic_bytes_per_layer": {
                "first": H * W * (4 + 4) + H * W * 64, "hidden": 2 * H * W * 64,
                "output": H * W * (64 + 4 + 4)}}


def run_train_step(args, spk, spkgen, torch, np):
    """The surrogate's graph-replayed training step alone, at the largest
    batch the plans take (64 crops of 128x128, 1 M px per step), on
    ``--sur-scenes`` static block scenes: 10 warm-up steps, then 30 timed."""
    import paper_2412_11639_amd.surrogate as sur
    B, Hc, Wc, n = 64, 128, 128, 40
    scenes = sur.SceneSet([10000 + i for i in range(args.sur_scenes)], H=250, W=400, T=4096,
                          keep_host=False)
    model = sur.Surrogate(seed=0)
    rng = np.random.default_rng(1)
    plan = sur.TrainPlan(model, [scenes.samples(rng, B, Hc, Wc) for _ in range(n)], [3e-4] * n,
                         Hc, Wc)
    plan.run(10)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    plan.run(n - 10)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / (n - 10)
    plan.close()
    tf = SUR_TRAIN_FLOP_PER_PX * B * Hc * Wc / (ms * 1e-3) / 1e12
    return {"batch": "%d crops of %dx%d" % (B, Hc, Wc), "ms_per_step": round(ms, 4),
            "tflops": round(tf, 2), "mfma_frac": round(tf / MFMA_BF16_PEAK_TFLOPS, 5)}


def run_encoded(args, spk, spkgen, torch, np):
    """The streaming scene's plain single pass (every frame from 31 on)
    and the same through segment lists + decode, nothing else."""
    H = W = 1000
    T = args.stream_frames
    s, speed, _, _ = _streaming_scene(spkgen, np, H, W, T)
    ds = torch.from_numpy(s).cuda()
    frames = list(range(31, T))
    out = torch.empty((len(frames), H, W), dtype=torch.float32, device="cuda")
    spk.reconstruct(ds, H, W, T, 1.0, frames, order=spk.FSR, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    spk.reconstruct(ds, H, W, T, 1.0, frames, order=spk.FSR, out=out)
    e1.record()
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1)
    idx = np.linspace(0, len(frames) - 1, 64).astype(int).tolist()
    kept = out[idx].cpu().numpy()
    res = {"workload": "blocks_1000x1000 translating |v|=%.3f px/frame (seed 5), %d frames"
                       % (speed, T),
           "plain_single_pass": {"mpx_frames_per_s": round(H * W * T / (plain_ms * 1e-3) / 1e6, 1),
                                 "ms": round(plain_ms, 3),
                                 "outputs": "every frame 31..%d" % (T - 1)},
           "plain_encoded": _encoded_leg(spk, torch, ds, H, W, T, frames, out, idx, kept),
           "plain_encoded_planar": _encoded_leg(spk, torch, ds, H, W, T, frames, out, idx, kept,
                                                packed=False)}
    del ds, out
    torch.cuda.empty_cache()
    return res


def run_streaming(args, spk, spkgen, torch, np, model, sur, static_model=None):
    """1000x1000 blocks translating at one velocity, |v| in (0, 2] px/frame
    (seed 5).  Per frame: advance the 32-frame window, run the surrogate
    (``model``, trained on moving scenes) and the fallback mux; latency from
    HIP events around each frame.  At the checked frames the network trained
    on static scenes (``static_model``) runs too, outside the timed region.
    Beside it the plain method two ways: one pass over the whole stream with
    an output every frame, and the latency-bound form that re-scans the last
    4096 frames for each output frame."""
    H = W = 1000
    T = args.stream_frames
    s, speed, vx, vy = _streaming_scene(spkgen, np, H, W, T)
    ds = torch.from_numpy(s).cuda()
    win = torch.zeros((1, H, W), dtype=torch.int32, device="cuda")
    est = torch.zeros((1, H, W), dtype=torch.float32, device="cuda")
    st = torch.zeros((1, H, W), dtype=torch.uint8, device="cuda")
    y = torch.empty((1, H, W), dtype=torch.float32, device="cuda")
    mx = torch.empty((1, H, W), dtype=torch.float32, device="cuda")
    n_check = min(400, T - 31)
    check_t = sorted(set(np.linspace(31, T - 1, n_check).astype(int).tolist()))
    names = ["surrogate", "surrogate_with_fallback", "plain_short_window"]
    if static_model is not None:
        names.append("surrogate_static_trained")
    kept = {k: torch.empty((len(check_t), H, W), dtype=torch.float32, device="cuda")
            for k in names}
    slot = {t: i for i, t in enumerate(check_t)}
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(T)]
    print("streaming: %d frames" % T, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for t in range(T):
        a, b = evs[t]
        a.record()
        sur.Surrogate.stream_step(ds[t], H, W, 1.0, win, est, st)
        if t >= 31:
            # the weights are packed once, by the first frame's inference
            model.infer(win, est, out=y, prepacked=t > 31)
            sur.Surrogate.mux(y, est, st, out=mx)
        b.record()
        if t in slot:
            kept["surrogate"][slot[t]].copy_(y[0])
            kept["surrogate_with_fallback"][slot[t]].copy_(mx[0])
            kept["plain_short_window"][slot[t]].copy_(est[0])
            if static_model is not None:
                static_model.infer(win, est, out=kept["surrogate_static_trained"][slot[t]][None])
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    lat = np.array([evs[t][0].elapsed_time(evs[t][1]) for t in range(31, T)])
    sur_rate = H * W * len(lat) / (lat.sum() * 1e-3) / 1e6
    fwd = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fwd[0].record()
    for _ in range(20):
        model.infer(win, est, out=y)
    fwd[1].record()
    torch.cuda.synchronize()
    fwd_ms = fwd[0].elapsed_time(fwd[1]) / 20
    fwd[0].record()
    for _ in range(20):
        model.infer(win, est, out=y, prepacked=True)
    fwd[1].record()
    torch.cuda.synchronize()
    fwd_pp_ms = fwd[0].elapsed_time(fwd[1]) / 20
    # plain, one pass, an output every frame from 31 on
    frames = list(range(31, T))
    plain_out = torch.empty((len(frames), H, W), dtype=torch.float32, device="cuda")
    spk.reconstruct(ds, H, W, T, 1.0, frames, order=spk.FSR, out=plain_out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    spk.reconstruct(ds, H, W, T, 1.0, frames, order=spk.FSR, out=plain_out)
    e1.record()
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1)
    plain_kept = plain_out[[t - 31 for t in check_t]].cpu().numpy()
    # the live form: the same stream fed 32 frames at a time (the paper's
    # hardware block), each pixel's state kept on the device between pieces,
    # the same every-frame outputs
    plain_out.fill_(-1.0)
    live = spk.Stream(H, W, 1.0, frames, order=spk.FSR, out=plain_out)
    torch.cuda.synchronize()
    e0.record()
    for a in range(0, T, 32):
        live.feed(ds[a:a + 32])
    live.finish()
    e1.record()
    torch.cuda.synchronize()
    live_ms = e0.elapsed_time(e1)
    live_same = bool(np.array_equal(plain_out[[t - 31 for t in check_t]].cpu().numpy(),
                                    plain_kept))
    live.close()
    # the same through the segment encoding: one pass writes each pixel's
    # segment list, a second expands it to every frame
    enc = _encoded_leg(spk, torch, ds, H, W, T, frames, plain_out,
                       [t - 31 for t in check_t], plain_kept)
    enc_planar = _encoded_leg(spk, torch, ds, H, W, T, frames, plain_out,
                              [t - 31 for t in check_t], plain_kept, packed=False)
    del plain_out
    # plain, latency-bound: re-scan the last Wn frames for one output frame
    Wn = min(4096, T)
    one = torch.empty((1, H, W), dtype=torch.float32, device="cuda")
    rs_ms = []
    for t in np.linspace(Wn - 1, T - 1, 8).astype(int):
        sub = ds[t - Wn + 1:t + 1]
        spk.reconstruct(sub, H, W, Wn, 1.0, [Wn - 1], order=spk.FSR, out=one)
        e0.record()
        spk.reconstruct(sub, H, W, Wn, 1.0, [Wn - 1], order=spk.FSR, out=one)
        e1.record()
        torch.cuda.synchronize()
        rs_ms.append(e0.elapsed_time(e1))
    rs_ms = float(np.median(rs_ms))
    res = {"workload": "blocks_1000x1000 translating |v|=%.3f px/frame (seed 5), %d frames"
                       % (speed, T),
           "frames": T,
           "surrogate_mpx_frames_per_s": round(sur_rate, 1),
           "latency_ms_p50": round(float(np.percentile(lat, 50)), 4),
           "latency_ms_p99": round(float(np.percentile(lat, 99)), 4),
           "surrogate_forward_ms": round(fwd_ms, 4),
           "surrogate_forward_prepacked_ms": round(fwd_pp_ms, 4),
           "surrogate_mfma_frac": round(SUR_FLOP_PER_PX * H * W / (fwd_pp_ms * 1e-3) / 1e12
                                        / MFMA_BF16_PEAK_TFLOPS, 4),
           "plain_single_pass": {"mpx_frames_per_s": round(H * W * T / (plain_ms * 1e-3) / 1e6, 1),
                                 "ms": round(plain_ms, 3),
                                 "outputs": "every frame 31..%d" % (T - 1)},
           "plain_live_32_frame_pieces": {
               "mpx_frames_per_s": round(H * W * T / (live_ms * 1e-3) / 1e6, 1),
               "ms": round(live_ms, 3), "pieces": (T + 31) // 32,
               "equals_single_pass": live_same},
           "plain_encoded": enc,
           "plain_encoded_planar": enc_planar,
           "plain_rescan_%d" % Wn: {"mpx_frames_per_s": round(H * W / (rs_ms * 1e-3) / 1e6, 1),
                                    "latency_ms": round(rs_ms, 4)},
           "wall_s": round(wall, 2)}
    check = dict(stream=s, H=H, W=W, T=T, times=check_t, plain=plain_kept,
                 **{k: v.cpu().numpy() for k, v in kept.items()})
    # the scene itself (the generator's per-frame intensity) as a third reference
    truth = spkgen.blocks_truth(H, W, check_t, 5, vx=vx, vy=vy)
    check["truth"] = truth
    res["vs_scene_truth_psnr_db"] = {k: round(_psnr(check[k], truth, np), 2) for k in names}
    res["vs_scene_truth_psnr_db"]["plain_whole_stream"] = round(_psnr(plain_kept, truth, np), 2)
    del ds, kept
    torch.cuda.empty_cache()
    return res, check


def run_accuracy(spk, spkgen, torch, np):
    """Synthetic analogue of the paper's quality comparison (Sec. IV):
    PSNR of FSR, SSR, the third order and the TFI / TFP baselines against
    the scene's true intensity (the generator's per-frame rate), at 16
    output frames."""
    H, W, T = 250, 400, 4096
    t_out = np.linspace(128, T - 1, 16).astype(int).tolist()
    scenes = {
        "static_blocks": (spkgen.blocks(H, W, T, 1),
                          lambda: spkgen.blocks_truth(H, W, t_out, 1)),
        "moving_blocks_v0.25": (spkgen.blocks(H, W, T, 4, vx=0.25, vy=0.1),
                                lambda: spkgen.blocks_truth(H, W, t_out, 4, vx=0.25, vy=0.1)),
        "gratings_poisson": (spkgen.gratings(H, W, T, 2),
                             lambda: spkgen.gratings_truth(H, W, t_out, 2)),
    }
    res = {}
    for name, (s, truth_fn) in scenes.items():
        ds = torch.from_numpy(s).cuda()
        truth = truth_fn()
        outs = {"FSR": spk.reconstruct(ds, H, W, T, 1.0, t_out, order=spk.FSR),
                "SSR": spk.reconstruct(ds, H, W, T, 1.0, t_out, order=spk.SSR),
                "third order": spk.reconstruct(ds, H, W, T, 1.0, t_out, order=spk.TSR),
                "TFI": spk.reconstruct(ds, H, W, T, 1.0, t_out, order=spk.TFI),
                "TFP-32": spk.tfp(ds, H, W, T, 1.0, 32, t_out),
                "TFP-64": spk.tfp(ds, H, W, T, 1.0, 64, t_out)}
        torch.cuda.synchronize()
        res[name] = {k: round(_psnr(v.cpu().numpy(), truth, np), 2) for k, v in outs.items()}
        del ds
    # static / motion mask (SSR, 64-frame window) on a scene whose left half
    # is the static blocks and right half the moving ones, against pixels
    # whose true intensity changed within the window
    half = W // 2
    bs = spkgen.unpack(scenes["static_blocks"][0], H, W)
    bm = spkgen.unpack(scenes["moving_blocks_v0.25"][0], H, W)
    bs[:, :, half:] = bm[:, :, half:]
    ds = torch.from_numpy(spkgen.pack(bs)).cuda()
    del bs, bm
    m = spk.motion(ds, H, W, T, 64, t_out, order=spk.SSR).cpu().numpy().astype(bool)
    prev_t = [t - 63 for t in t_out]
    tm = scenes["moving_blocks_v0.25"][1]()
    moved = tm != spkgen.blocks_truth(H, W, prev_t, 4, vx=0.25, vy=0.1)
    moved[:, :, :half] = False
    tp = int((m & moved).sum())
    res["motion_mask"] = {
        "scene": "left half static blocks, right half moving blocks; SSR, window 64",
        "precision": round(tp / max(1, int(m.sum())), 4),
        "recall": round(tp / max(1, int(moved.sum())), 4),
        "static_half_flagged": round(float(m[:, :, :half].mean()), 5)}
    del ds
    return {"workload": "250x400x4096 scenes, 16 outputs t=128..4095, PSNR (dB, peak 1) "
                        "against the generator's true intensity", "psnr_db": res}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


CPU_RUNS = 9  # timed oracle runs for the cpu_baseline figure (about 10 s on 16 threads)


def cpu_baseline_leg(args, plain, batched, sur_checks, res, np):
    """Every use of the oracle in this benchmark.  Times the oracle on a
    sample of the plain workload (the cpu_baseline figure) and checks the
    GPU outputs of every leg against it: bit-exact for the plain method,
    PSNR and maximum absolute error for the surrogate."""
    import oracle
    import spkgen
    nproc = len(os.sched_getaffinity(0))
    # one GPU's share of the host is 16 cores: never more threads than that
    n = min(16, nproc)
    s, H, W, T, t_out, order, gpu_out = plain
    rows = min(args.cpu_rows, H)
    print("cpu baseline: oracle on %d rows" % rows, file=sys.stderr, flush=True)
    sub = s if rows == H else spkgen.pack(spkgen.unpack(s, H, W)[:, :rows, :])
    oracle.reconstruct(sub[:256], rows, W, 256, 1.0, [0], order=order, nthreads=n)  # warm
    runs = []
    for _ in range(CPU_RUNS):
        t0 = time.perf_counter()
        ref = oracle.reconstruct(sub, rows, W, T, 1.0, t_out, order=order, nthreads=n)
        runs.append(time.perf_counter() - t0)
    dt = float(np.median(runs))
    ok = bool(np.array_equal(gpu_out[:, :rows, :], ref.astype(np.float32)))
    del ref
    r1 = min(16, rows)
    sub1 = spkgen.pack(spkgen.unpack(s, H, W)[:, :r1, :])
    t0 = time.perf_counter()
    oracle.reconstruct(sub1, r1, W, T, 1.0, t_out, order=order, nthreads=1)
    dt1 = time.perf_counter() - t0
    res["cpu_baseline"] = {
        "value": round(rows * W * T / dt / 1e6, 1), "unit": "Mpixel-frames/s", "cores": n,
        "nproc": nproc, "cpu_model": _cpu_model(), "kind": "oracle",
        "sample": "%d of %d rows, all %d frames and %d outputs (%s); median of %d runs "
                  "(%.2f s each) after a warm-up; GPU output on the same rows bit-exact: %s"
                  % (rows, H, T, len(t_out), "SSR" if order == 2 else "FSR", CPU_RUNS, dt, ok),
        "single_thread_value": round(r1 * W * T / dt1 / 1e6, 2)}
    failures = [] if ok else ["plain"]
    if batched is not None:
        j = batched["job"]
        r = oracle.reconstruct(batched["stream"], j["H"], j["W"], j["T"], 1.0, j["t_out"],
                               order=batched["order"], nthreads=n)
        eq = bool(np.array_equal(batched["got"], r.astype(np.float32)))
        res["batched"]["smallest_stream_bit_exact_vs_oracle"] = eq
        failures += [] if eq else ["batched"]
    if sur_checks:
        c = sur_checks["surrogate"]
        refs = np.concatenate([oracle.reconstruct(h, c["H"], c["W"], c["T"], 1.0, c["times"],
                                                  order=1, nthreads=n) for h in c["host"]])
        eq = bool(np.array_equal(c["plain_long"], refs.astype(np.float32)))
        res["surrogate"]["vs_oracle"] = {
            "psnr_db": {"surrogate": round(_psnr(c["y"], refs, np), 2),
                        "surrogate_with_fallback": round(_psnr(c["mux"], refs, np), 2),
                        "plain_short_window": round(_psnr(c["est"], refs, np), 2)},
            "max_abs": {"surrogate": float("%.4g" % np.abs(c["y"] - refs).max()),
                        "surrogate_with_fallback": float("%.4g" % np.abs(c["mux"] - refs).max()),
                        "plain_short_window": float("%.4g" % np.abs(c["est"] - refs).max())},
            "training_targets_bit_exact": eq}
        failures += [] if eq else ["surrogate targets"]
        c = sur_checks["streaming"]
        print("cpu leg: streaming references at %d frames" % len(c["times"]),
              file=sys.stderr, flush=True)
        refs = oracle.reconstruct(c["stream"], c["H"], c["W"], c["T"], 1.0, c["times"],
                                  order=1, nthreads=n)
        eq = bool(np.array_equal(c["plain"], refs.astype(np.float32)))
        q = {"frames": len(c["times"]), "plain_bit_exact": eq}
        for name, r in (("whole_stream", refs), ("causal", None)):
            if r is None:
                r = oracle.reconstruct(c["stream"], c["H"], c["W"], c["T"], 1.0, c["times"],
                                       order=1, nthreads=n, causal=True)
            keys = [k for k in ("surrogate", "surrogate_with_fallback", "plain_short_window",
                                "surrogate_static_trained") if k in c]
            q[name] = {"psnr_db": {k: round(_psnr(c[k], r, np), 2) for k in keys},
                       "max_abs": {k: float("%.4g" % np.abs(c[k] - r).max()) for k in keys}}
            if name == "causal":
                res["streaming"]["vs_scene_truth_psnr_db"]["plain_causal"] = round(
                    _psnr(r, c["truth"], np), 2)
                # how close the method itself comes, on all frames up to t,
                # to its whole-stream output: a causal reference point for
                # any estimator that sees only the past
                q["causal_oracle_vs_whole_stream_psnr_db"] = round(_psnr(r, whole, np), 2)
                del whole
            else:
                whole = r
            del r
        del refs
        res["streaming"]["vs_oracle"] = q
        failures += [] if eq else ["streaming plain"]
    return failures


def parse_rocprof(d: str) -> str:
    """Summarise rocprofv3 output (rocpd SQLite databases or CSV) under d."""
    import sqlite3
    lines = []
    for f in sorted(glob.glob(os.path.join(d, "**", "*_results.db"), recursive=True)):
        con = sqlite3.connect(f)
        lines.append("# rocpd: %s" % os.path.relpath(f, d))
        try:
            for name, calls, total, avg in con.execute(
                    "select name, total_calls, total_duration, average from top_kernels"):
                lines.append("kernel %-70s calls=%-5d avg_ns=%-12.1f total_ns=%.1f"
                             % (name[:70], calls, avg, total))
        except sqlite3.Error:
            pass
        try:
            for name, cname, n, mean in con.execute(
                    "select kernel_name, counter_name, count(*), avg(value) "
                    "from counters_collection group by kernel_name, counter_name"):
                lines.append("counter %-70s %-12s dispatches=%-4d mean=%.1f"
                             % (name[:70], cname, n, mean))
        except sqlite3.Error:
            pass
        con.close()
    stats = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)
    for f in stats:
        lines.append("# kernel stats: %s" % os.path.relpath(f, d))
        with open(f) as fh:
            rows = list(csv.DictReader(fh))
        for r in rows:
            lines.append("%-60s calls=%-6s avg_ns=%-12s total_ns=%-14s pct=%s" % (
                r.get("Name", "")[:60], r.get("Calls"), r.get("AverageNs"),
                r.get("TotalDurationNs"), r.get("Percentage")))
    pmc = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    for f in pmc:
        lines.append("# counters: %s" % os.path.relpath(f, d))
        agg = {}
        with open(f) as fh:
            for r in csv.DictReader(fh):
                key = (r.get("Kernel_Name", "")[:60], r.get("Counter_Name"))
                agg.setdefault(key, []).append(float(r.get("Counter_Value", 0)))
        for (k, c), v in sorted(agg.items()):
            lines.append("%-60s %-12s dispatches=%-5d mean=%.1f" % (k, c, len(v), sum(v) / len(v)))
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--order", choices=["fsr", "ssr"], default="ssr")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=250,
                    help="rows of the plain workload the oracle runs on (all by default)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (counter calibration)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched 16-stream measurement")
    ap.add_argument("--only-batched", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip surrogate training/evaluation and the streaming run")
    ap.add_argument("--only-surrogate", action="store_true")
    ap.add_argument("--only-forward", action="store_true",
                    help="only the surrogate forward at 1000x1000")
    ap.add_argument("--only-train-step", action="store_true",
                    help="only the surrogate training step at 64 crops of 128x128")
    ap.add_argument("--only-encoded", action="store_true",
                    help="only the streaming scene's single pass and segment lists + decode")
    ap.add_argument("--no-other-paths", action="store_true",
                    help="skip timing the third order, TFI, TFP-32 and the motion mask")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the FSR/SSR/TFI/TFP quality comparison")
    ap.add_argument("--sur-steps", type=int, default=3000)
    ap.add_argument("--sur-scenes", type=int, default=256)
    ap.add_argument("--sur-moving-scenes", type=int, default=128)
    ap.add_argument("--stream-frames", type=int, default=40000,
                    help="frames of the 1000x1000 streaming run (the configuration's 40000)")
    ap.add_argument("--parse-rocprof", default=None)
    ap.add_argument("--traffic-out", default=None,
                    help="with --parse-rocprof: write the per-launch HBM traffic JSON")
    args = ap.parse_args()

    if args.parse_rocprof:
        print(parse_rocprof(args.parse_rocprof))
        if args.traffic_out:
            t = {"kernel_sha": kernel_sha(), "per_order": traffic_from_counters(args.parse_rocprof),
                 "note": "FETCH_SIZE and WRITE_SIZE (KiB per dispatch) scaled by the same "
                         "counter's reading for a 1 GiB device copy"}
            with open(args.traffic_out, "w") as f:
                json.dump(t, f, indent=1)
        return 0
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2412_11639_amd as spk
    import spkgen

    if (args.only_batched or args.only_surrogate or args.only_encoded or args.only_forward
            or args.only_train_step):
        args.no_cpu_baseline = True
        out = {}
        if args.copy_calibration:
            a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
            b = torch.empty_like(a)
            b.copy_(a)
            torch.cuda.synchronize()
            del a, b
        if args.only_encoded:
            out["encoded"] = run_encoded(args, spk, spkgen, torch, np)
        if args.only_forward:
            out["forward"] = run_forward(args, spk, spkgen, torch, np)
        if args.only_train_step:
            out["train_step"] = run_train_step(args, spk, spkgen, torch, np)
        if args.only_batched:
            out["batched"] = run_batched(args, spk, spkgen, torch, np)[0]
        if args.only_surrogate:
            out.update(run_surrogate(args, spk, spkgen, torch, np)[0])
        print(json.dumps(out))
        return 0

    wl = spkgen.GRATINGS_250x400
    H, W, T = wl.H, wl.W, wl.T
    t_out = wl.times()
    n_out = len(t_out)
    order = spk.SSR if args.order == "ssr" else spk.FSR
    print("generating %s" % wl.name, file=sys.stderr, flush=True)
    s = wl.generate()
    ds = torch.from_numpy(s).cuda()
    out = torch.empty((n_out, H, W), dtype=torch.float32, device="cuda")

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    def step(o=order):
        spk.reconstruct(ds, H, W, T, 1.0, t_out, order=o, out=out)

    def timed(o):
        for _ in range(args.warmup):
            step(o)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        w0 = time.perf_counter()
        e0.record()
        for _ in range(args.steps):
            step(o)
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        return e0.elapsed_time(e1) / args.steps, wall

    def copy_bandwidth():
        # a 1 GiB device-to-device copy: bytes read + written per second
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        c0.record()
        for _ in range(5):
            b.copy_(a)
        c1.record()
        torch.cuda.synchronize()
        ms_copy = c0.elapsed_time(c1) / 5
        del a, b
        torch.cuda.empty_cache()
        return 2.0 * COPY_BYTES / (ms_copy * 1e-3) / 1e9

    print("timing %d steps" % args.steps, file=sys.stderr, flush=True)
    other = spk.FSR if order == spk.SSR else spk.SSR
    ms_other, _ = timed(other)
    ms, wall = timed(order)
    gpu_out = out.cpu().numpy()

    px_frames = H * W * T
    value = px_frames / (ms * 1e-3) / 1e6
    alg = algorithmic_bytes(H, W, T, n_out)
    achieved = alg / (ms * 1e-3) / 1e9
    copy_gbs = copy_bandwidth()
    counters = load_counters(args.order.upper())
    traffic = counters.get("hbm_bytes_per_launch")
    traffic = None if traffic is None else round(traffic)
    valu = counters.get("valu_per_launch")

    res = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "Mpixel-frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": wl.name, "H": H, "W": W, "T": T, "n_out": n_out,
                   "order": args.order.upper(), "theta": 1.0,
                   "scene": "1-3 moving sinusoidal gratings + rotating sectored disk, "
                            "Poisson photons (1000 per threshold), seed 2"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic},
        "hbm_copy": {"GBs": round(copy_gbs, 1),
                     "what": "1 GiB device-to-device copy, bytes read + written per second",
                     "achieved_frac_of_copy": round(achieved / copy_gbs, 4)},
        "valu": None if valu is None else {
            "note": "the kernel is bound by integer VALU issue, not HBM",
            "instr_per_step": round(valu), "issue_per_s": round(valu / (ms * 1e-3)),
            "peak_per_s": VALU_PEAK_PER_S, "frac": round(valu / (ms * 1e-3) / VALU_PEAK_PER_S, 3)},
        "cpu_baseline": None,
        "other_order": {"order": "FSR" if order == spk.SSR else "SSR",
                        "ms_per_step": round(ms_other, 4),
                        "value": round(px_frames / (ms_other * 1e-3) / 1e6, 1)},
        "wall_s_timed": round(wall, 3),
    }
    if not args.no_other_paths:
        res["other_paths"] = other_paths(spk, torch, ds, H, W, T, t_out, out)
        res["small_static"] = run_small(spk, spkgen, torch, np)
    del ds, out
    torch.cuda.empty_cache()
    bcheck, schecks = None, None
    if not args.no_batched:
        res["batched"], bcheck = run_batched(args, spk, spkgen, torch, np)
    if not args.no_accuracy:
        print("accuracy: FSR / SSR / TFI / TFP against scene truth", file=sys.stderr, flush=True)
        res["accuracy"] = run_accuracy(spk, spkgen, torch, np)
    if not args.no_surrogate:
        sres, schecks = run_surrogate(args, spk, spkgen, torch, np)
        res.update(sres)
    if not args.no_cpu_baseline:
        failures = cpu_baseline_leg(args, (s, H, W, T, t_out, order, gpu_out), bcheck, schecks,
                                    res, np)
        if failures:
            print("PARITY FAILURE against the oracle: %s" % ", ".join(failures), file=sys.stderr)
            print(json.dumps(res))
            return 1
    print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
