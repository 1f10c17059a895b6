"""Benchmark of the MAFOD hot path on one MI355X.

A step is one mf4d_filter call over the roofline-scale workload: a 4096 x 4096
float32 image with 64 bright and dark creases (widths 1-16 px, noise
N(0, 0.05)), 8 log-spaced scales 1..16, ridge+valley mode, 30 FED cycles of
20 substeps -- scale selection, normalised Hessian and every substep included,
with the input already resident in HBM. The call is recorded once into a
hipGraph and each step replays it (the same kernels and launch shapes as the
eager call, which gives the same bits); --eager times the call itself, and
the graph run reports the eager time beside it.

Prints one JSON line:
  value     Mpixel-FED-substeps/s of the whole filter (H W M n per step / time)
  roofline  the fused FED substep kernel as the filter launches it (4 substeps
            per launch): algorithmic bytes per launch (20 B/px: u read 4,
            tensor planes read 12, u write 4) / its average launch time,
            timed with HIP events on the stream it is launched on, against
            the 8 TB/s HBM peak
  roofline_alu  the same launches in FP32 vector flops (37 per px-substep)
  roofline_selection  scale sweep, argmax and integration (rows a2-a4) per
            cycle: 26 B/px algorithmic (sweep and argmax: u read twice, as the
            image-wide c needs every scale before any argmax, 8, index
            written 1; integration: u 4 and index 1 read, tensor planes
            written 12) over the filter's per-cycle time outside its
            substep launches
  roofline_sweep  the fused scale-sweep kernel at sigma = 16 (both separable
            passes of one scale on the matrix cores, split-BF16 products):
            algorithmic flops (8 filters x 99 taps x 2 per pixel) against the
            FP32-equivalent peak of split-BF16 products (BF16 peak / 6)
  hbm_copy_probe  a plain 1 GiB device copy: the HBM rate the box reaches in practice
  cpu_baseline  the FP64 oracle on a bounded sample (the first 3 cycles of the same image)
  extensions  batched_256 (256 uneven images in one batch plan vs per-image
            calls), learned_2048 (the learned selection vs the exact sweep),
            volume_256 (the filter on a 256^3 volume) and aux_4096 (scale-image
            postprocessing, l2-optimal stopping, crease extraction and matching
            on the 4096^2 image)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # B/s, MI355X HBM3E
# FP32 vector peak without packed FP32: 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
VALU_PEAK = 78.6e12        # FLOP/s
MFMA_F32_PEAK = 157.3e12   # FLOP/s, dense FP32 matrix cores
MFMA_BF16_PEAK = 2.5e15    # FLOP/s, dense BF16 matrix cores
BF3_PRODUCTS = 6           # BF16 part products per FP32 product in the split-BF16 sweep
SUBSTEP_BYTES_PER_PX = 20  # per launch: u in 4 + tensor planes in 12 + u out 4
SUBSTEP_FLOPS_PER_PX = 37  # per substep: L u 10, D L u 13, L^T and update 14
SUBSTEPS_PER_LAUNCH = 4    # as mf4d_filter launches the fused substep kernel (two columns per lane)
# rows a2-a4 per pixel and cycle: sweep and argmax 9 (u read twice, since the
# image-wide c needs every scale before any argmax, 8; index written 1) and
# integration 17 (u 4 and index 1 read, tensor planes written 12)
SELECTION_BYTES_PER_PX = 26
CPU_CYCLES = 3             # FED cycles of the oracle's bounded sample (about 15 s on 16 host cores)


CSRC = os.path.join(ROOT, "paper_1611_06906_amd", "csrc")
# sources whose change invalidates a kernel's committed counter figures
KERNEL_SOURCES = {
    "fed_stream2_kernel<4>": ["fed_kernels.hip", "fed_tiles.h", "mf4d_internal.h", "../build.py"],
    "sweep_fused_kernel<8>": ["scale_kernels.hip", "scale_mfma.h", "scale_tiles.h", "mf4d_internal.h", "../build.py"],
    "fed3_kernel": ["vol3d.hip", "mf4d_internal.h", "../build.py"],
}


def source_digest(kernel):
    """sha256 prefix over the sources of `kernel` (in KERNEL_SOURCES order)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()[:16]


def trace_mean_us(kernel, row):
    """Mean duration (us) of the summary row `row` of `kernel` in the committed
    kernel trace, or None if the kernel's sources changed since it was taken."""
    prof = os.path.join(ROOT, "profiles", "creases4096_kernel_trace.txt")
    try:
        text = open(prof).read()
        digest = source_digest(kernel)
    except (OSError, KeyError):
        return None
    if f"{kernel} sources sha256 prefix: {digest}" not in text:
        return None
    for line in text.splitlines():
        if line.startswith(row + " "):
            nums = line[len(row):].split()   # count, mean, min, max, total
            try:
                return float(nums[1])
            except (IndexError, ValueError):
                return None
    return None


def counter_traffic(kernel, row=None, summary="creases4096_hbm_counters.txt"):
    """HBM bytes per launch of `kernel` (its summary row `row`, default the
    kernel itself) from the committed rocprofv3 counter summary `summary`
    (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, calibrated on a plain copy), or
    None if the kernel's sources changed since the counters were taken."""
    prof = os.path.join(ROOT, "profiles", summary)
    try:
        text = open(prof).read()
        digest = source_digest(kernel)
    except (OSError, KeyError):
        return None
    if f"{kernel} sources sha256 prefix: {digest}" not in text:
        return None
    row = row or kernel
    for line in text.splitlines():
        if "sha256" in line or not (line.startswith(row + " ") or line.startswith("void " + row + " ")):
            continue
        cols = line.split()
        nums = [c for c in cols if c.replace(".", "", 1).isdigit()]
        try:   # n, FETCH_KiB, WRITE_KiB, read_MB, write_MB, ...
            return (float(nums[3]) + float(nums[4])) * 1e6
        except (IndexError, ValueError):
            return None
    return None


def selection_traffic():
    """HBM bytes of one cycle's scale sweep, argmax and integration from the
    committed counter summary: the sum of per_cycle x (read_MB + write_MB)
    over its rows of stage "sel", or None if absent or stale."""
    prof = os.path.join(ROOT, "profiles", "creases4096_hbm_counters.txt")
    try:
        text = open(prof).read()
        digest = source_digest("sweep_fused_kernel<8>")
    except (OSError, KeyError):
        return None
    if f"sweep_fused_kernel<8> sources sha256 prefix: {digest}" not in text:
        return None
    total, rows = 0.0, 0
    for line in text.splitlines():
        cols = line.split()
        if "sha256" in line or " sel " not in line or not cols or "_kernel" not in cols[0]:
            continue
        nums = [c for c in cols if c.replace(".", "", 1).isdigit()]
        try:   # n, FETCH_KiB, WRITE_KiB, read_MB, write_MB, per_cycle, ...
            total += int(nums[5]) * (float(nums[3]) + float(nums[4])) * 1e6
            rows += 1
        except (IndexError, ValueError):
            return None
    return total if rows else None


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def time_stream(torch, fn, reps):
    """Average ms of fn() over reps calls, HIP events on the current stream."""
    s, e = _events(torch)
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def _batch_image(spec):
    from paper_1611_06906_amd import synth
    return synth.batch_image(spec)


def batched_comparison(torch, mf4d, synth, dev, reps=2):
    """256 uneven images (sizes U[256, 1536], ridge/valley, cycles U[5, 25],
    scales 1, 1.5, 2, 3, n = 10): one batched graph vs per-image calls."""
    import numpy as np
    from concurrent.futures import ProcessPoolExecutor
    specs = synth.batch_of_images()
    t0 = time.time()
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with ProcessPoolExecutor(workers) as ex:
        imgs = list(ex.map(_batch_image, specs, chunksize=4))
    print(f"[bench] batch of {len(imgs)} images generated in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    sig = [1.0, 1.5, 2.0, 3.0]
    params = [mf4d.Params(sig, mode=sp["mode"], cycles=sp["cycles"], substeps=10) for sp in specs]
    shapes = [(sp["H"], sp["W"]) for sp in specs]
    packed = torch.from_numpy(np.concatenate([im.ravel() for im in imgs])).to(dev)
    out_b = torch.empty_like(packed)
    plan = mf4d.Batch(shapes, params)
    ws_b = plan.workspace(dev)
    t1 = time.time()
    plan.autotune(ws_b)
    tune = plan.tuning()
    plan.filter(packed, out_b, ws_b)          # records the graph
    torch.cuda.synchronize()
    print(f"[bench] batch autotune {tune}, setup {time.time() - t1:.1f}s", file=sys.stderr, flush=True)
    ms_b = time_stream(torch, lambda: plan.filter(packed, out_b, ws_b), reps)
    # per-image plain launches over the same images
    offs = np.concatenate([[0], np.cumsum([h * w for h, w in shapes])])
    views_in = [packed[offs[i]:offs[i + 1]].view(shapes[i]) for i in range(len(shapes))]
    out_p = torch.empty_like(packed)
    views_out = [out_p[offs[i]:offs[i + 1]].view(shapes[i]) for i in range(len(shapes))]
    big = max(mf4d.mf4d_workspace_bytes(h, w, p) for (h, w), p in zip(shapes, params))
    ws_p = torch.empty(big, dtype=torch.uint8, device=dev)

    def plain():
        for vi, vo, p in zip(views_in, views_out, params):
            mf4d.mf4d_filter(vi, vo, p, ws_p)

    plain()
    ms_p = time_stream(torch, plain, reps)
    torch.cuda.synchronize()
    same = bool(torch.equal(out_b, out_p))
    # the same per-image calls recorded once into one hipGraph and replayed:
    # per-image launches without the host's launch cost
    ms_pg = None
    try:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            plain()
        graph.replay()
        ms_pg = time_stream(torch, graph.replay, reps)
        same = same and bool(torch.equal(out_b, out_p))
        del graph
    except RuntimeError as e:
        print(f"[bench] per-image graph not recorded: {e}", file=sys.stderr, flush=True)
    px_sub = sum(h * w * sp["cycles"] * 10 for (h, w), sp in zip(shapes, specs))
    plan.close()
    return {"images": len(imgs), "megapixels": float(offs[-1]) / 1e6,
            "batched_ms": ms_b, "plain_ms": ms_p,
            "batched_images_per_s": len(imgs) / (ms_b * 1e-3), "plain_images_per_s": len(imgs) / (ms_p * 1e-3),
            "batched_Mpx_substeps_per_s": px_sub / (ms_b * 1e-3) / 1e6,
            "plain_Mpx_substeps_per_s": px_sub / (ms_p * 1e-3) / 1e6,
            "speedup": ms_p / ms_b, "bit_identical_to_plain": same,
            "plain_graph_ms": ms_pg,
            "plain_graph_images_per_s": (len(imgs) / (ms_pg * 1e-3)) if ms_pg else None,
            "speedup_vs_plain_graph": (ms_pg / ms_b) if ms_pg else None,
            "substeps_per_launch": tune[0], "rows_per_wave": tune[1]}


# one substep of the volume filter moves u in (4 B), the tensor (the six
# entries of the symmetric P: 24 B) and u out (4 B) per voxel
VOLUME_SUBSTEP_BYTES = 32


def volume_comparison(torch, mf4d, synth, dev, reps=3):
    """The filter on a 256^3 volume of 24 bright and dark tubes (widths
    U[1, 3]), 4 scales 1..3.375, both modes, 2 cycles of 10 substeps at
    tau_max = 1/27: voxel throughput and the substep kernels' HBM rate."""
    D = H = W = 256
    t0 = time.time()
    v = synth.tubes3d(D, H, W, 24, seed=0, signs="mixed", width_range=(1.0, 3.0))
    print(f"[bench] volume {D}x{H}x{W} generated in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    sig = [1.5 ** k for k in range(4)]
    cycles, n = 2, 10
    p = mf4d.Params(sig, mode=mf4d.MF4D_BOTH, cycles=cycles, substeps=n, tau_max=1.0 / 27.0)
    ui = torch.from_numpy(v).to(dev)
    uo = torch.empty_like(ui)
    ws = mf4d.workspace3(D, H, W, p, dev)
    run = lambda: mf4d.mf4d3d_filter(ui, uo, p, ws)
    run()
    ms = time_stream(torch, run, reps)
    # the substeps alone, from one cycle's tensor
    m = D * H * W
    idx = torch.empty((D, H, W), dtype=torch.uint8, device=dev)
    hr = torch.empty((6, D, H, W), dtype=torch.float32, device=dev)
    dp = torch.empty((D, H, W, 6), dtype=torch.float32, device=dev)
    mf4d.mf4d3d_scale_select(ui, p, idx, None, None, ws)
    mf4d.mf4d3d_tensor(ui, idx, p, hr, dp, ws)
    taus = mf4d.mf4d_fed_plan(p)[1]
    uc = ui.clone()
    ut = torch.empty_like(uc)
    # an even number of substeps ends in uc: the timing holds only the substep kernel
    cyc = lambda: mf4d.mf4d3d_fed_cycle_tensor(uc, dp, taus, ut)
    cyc()
    ms_sub = time_stream(torch, cyc, reps) / n
    t = ms_sub * 1e-3
    return {"volume": [D, H, W], "scales": sig, "cycles": cycles, "substeps": n,
            "filter_ms": ms, "Mvoxel_substeps_per_s": m * cycles * n / (ms * 1e-3) / 1e6,
            "ms_per_substep": ms_sub, "per_cycle_outside_substeps_ms": ms / cycles - n * ms_sub,
            "substep_roofline": {"bound": "hbm", "achieved": VOLUME_SUBSTEP_BYTES * m / t / 1e9,
                                 "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                                 "frac": VOLUME_SUBSTEP_BYTES * m / t / HBM_PEAK,
                                 "bytes_per_voxel": VOLUME_SUBSTEP_BYTES,
                                 "traffic": counter_traffic("fed3_kernel", summary="volume256_hbm_counters.txt"),
                                 "kernel": "fed3_kernel (fused substep, 32 x 8 tiles streaming along z)"}}


def _centreline_segments(lines):
    """Ground-truth segments between consecutive centreline samples of the
    generator's creases, as the matching takes them: (segs [n][4] as
    (x0, y0, x1, y1), types [n] = the crease's sign)."""
    import numpy as np
    segs, types = [], []
    for pts, sgn in lines:
        pts = np.asarray(pts, np.float32)
        if len(pts) >= 2:
            segs.append(np.concatenate([pts[:-1], pts[1:]], axis=1))
            types.append(np.full(len(pts) - 1, int(sgn), np.int32))
    return np.ascontiguousarray(np.concatenate(segs)), np.ascontiguousarray(np.concatenate(types))


def aux_comparison(torch, mf4d, synth, dev, reps=3, cycles=2):
    """The paper's further steps on the 4096^2 creases image, each timed with
    HIP events on the library's calls: scale-image postprocessing (Sec. 3.3,
    theta = 0.13) and l2-optimal stopping against the noise-free image
    (Sec. 4), as their cost per FED cycle over the plain filter (`cycles`
    cycles of 20 substeps); crease extraction (Sec. 3.6) on the filtered
    image and the matching of the ground-truth centreline segments (Sec. 4)
    to its segments."""
    import numpy as np
    w = synth.creases4096()
    t0 = time.time()
    img, clean, lines = w.ground_truth()
    print(f"[bench] aux: {w.name} with ground truth generated in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)
    H, W = w.H, w.W
    u = torch.from_numpy(img).to(dev)
    gt = torch.from_numpy(clean).to(dev)
    out = torch.empty_like(u)
    p = mf4d.Params.from_workload(w, cycles=cycles)
    pp = mf4d.Params.from_workload(w, cycles=cycles, postprocess=1, theta=0.13)
    ws = mf4d.workspace(H, W, pp, dev)
    l2 = torch.empty(cycles + 1, dtype=torch.float64, device=dev)
    best = torch.empty(1, dtype=torch.int32, device=dev)
    runs = {"plain": lambda: mf4d.mf4d_filter(u, out, p, ws),
            "postprocess": lambda: mf4d.mf4d_filter(u, out, pp, ws),
            "l2stop": lambda: mf4d.mf4d_filter_l2stop(u, out, p, gt, l2, best, ws)}
    ms = {}
    for k, f in runs.items():
        f()
        ms[k] = time_stream(torch, f, reps)
    # extraction and matching on the plainly filtered image
    runs["plain"]()
    cws = torch.empty(int(mf4d.lib().mf4d_creases_workspace_bytes(H, W)), dtype=torch.uint8, device=dev)
    seg = torch.empty((H - 1, W - 1, 2, 4), dtype=torch.float32, device=dev)
    typ = torch.empty((H - 1, W - 1, 2), dtype=torch.int8, device=dev)
    cre = lambda: mf4d.mf4d_creases(out, 1.0, 0.005, mf4d.MF4D_BOTH, seg, typ, ws=cws)
    cre()
    ms_cre = time_stream(torch, cre, reps)
    gs, gt_types = _centreline_segments(lines)
    gs_d, gtt_d = torch.from_numpy(gs).to(dev), torch.from_numpy(gt_types).to(dev)
    dist = torch.empty(len(gs), dtype=torch.float32, device=dev)
    match = torch.empty(len(gs), dtype=torch.int32, device=dev)
    mat = lambda: mf4d.mf4d_crease_match(seg, typ, gs_d, gtt_d, 6.0, dist, match)
    mat()
    ms_mat = time_stream(torch, mat, reps)
    torch.cuda.synchronize()
    matched = float((match >= 0).float().mean().item())
    # extraction reads u (4 B) and writes two segments and their types per cell (34 B)
    cre_bytes = 4 * H * W + 34 * (H - 1) * (W - 1)
    return {"image": [H, W], "cycles": cycles, "substeps": w.substeps,
            "plain_filter_ms": ms["plain"],
            "postprocess": {"filter_ms": ms["postprocess"],
                            "ms_per_cycle_over_plain": (ms["postprocess"] - ms["plain"]) / cycles, "theta": 0.13},
            "l2stop": {"filter_ms": ms["l2stop"], "ms_per_cycle_over_plain": (ms["l2stop"] - ms["plain"]) / cycles,
                       "best_cycle": int(best.item())},
            "creases": {"ms": ms_cre, "Mpx_per_s": H * W / (ms_cre * 1e-3) / 1e6,
                        "algorithmic_GBs": cre_bytes / (ms_cre * 1e-3) / 1e9,
                        "frac_hbm": cre_bytes / (ms_cre * 1e-3) / HBM_PEAK},
            "match": {"ms": ms_mat, "gt_segments": len(gs), "matched_share": matched}}


def _pool_image(args):
    """Training pool and test images of the learned comparison: fundus-type
    (config-2 recipe) or ridge-type (config-1 recipe, inverted so that its
    creases are valleys like the vessels the valley-mode scales select)."""
    from paper_1611_06906_amd import synth
    H, seed, ridges = args
    if ridges:
        u = synth.creases(H, H, max(1, round(3 * H / 128)), seed)
        return (1.0 - u.astype("float64")).astype("float32")
    return synth.fundus(H, H, seed)


def learned_comparison(torch, mf4d, synth, dev, patches=20000, batch=16, reps=1):
    """Learned scale surrogate vs the plain filter on four 2048 x 2048
    fundus-like images (8 scales 8^(k/7), valley mode, 20 FED cycles x 15,
    confidence threshold 0.9). The network is first trained here, on the GPU
    with the library's kernels: `patches` random 256 x 256 crops (half of
    fundus type, half of ridge type) drawn from a pool of 64 images of
    1024 x 1024, labelled by the exact sweep, one pass in batches of
    `batch`. Accuracy against the oracle is the business of the tests (the learned filter against its
    oracle); here the learned filter's final images are compared with the
    plain filter's; an untrained network gives the ablation."""
    import numpy as np
    from concurrent.futures import ProcessPoolExecutor
    sig = [8.0 ** (k / 7.0) for k in range(8)]
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    t0 = time.time()
    jobs = [(1024, 10000 + i, i >= 32) for i in range(64)] + [(2048, 50000 + i, False) for i in range(4)]
    with ProcessPoolExecutor(workers) as ex:
        imgs = list(ex.map(_pool_image, jobs, chunksize=2))
    pool, test_imgs = imgs[:64], imgs[64:]
    print(f"[bench] learned: images generated in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    psel = mf4d.Params(sig, mode=mf4d.MF4D_VALLEY)
    U = torch.stack([torch.from_numpy(u).to(dev) for u in pool])
    L = torch.empty(U.shape, dtype=torch.uint8, device=dev)
    ws_sel = mf4d.workspace(1024, 1024, psel, dev)
    for i in range(len(pool)):
        mf4d.mf4d_scale_select(U[i], psel, L[i], None, None, ws_sel)
    del ws_sel
    th = mf4d.net_init(0, dev)
    th0 = th.clone()
    g = torch.zeros_like(th)
    mm, vv = torch.zeros_like(th), torch.zeros_like(th)
    stats = torch.zeros(2, dtype=torch.float32, device=dev)
    B, C = batch, 256
    steps = patches // B
    ws = mf4d.net_workspace(B, C, C, True, dev)
    rng = np.random.default_rng(0)
    torch.cuda.synchronize()
    t1 = time.time()
    ar = torch.arange(C, device=dev)
    half = len(pool) // 2
    for step in range(1, steps + 1):
        # the step's crops, half from each image type, in one gather per tensor
        which = np.concatenate([rng.integers(0, half, B // 2), rng.integers(half, len(pool), B - B // 2)])
        sel = torch.from_numpy(np.stack([which, rng.integers(0, 1024 - C + 1, B),
                                         rng.integers(0, 1024 - C + 1, B)])).to(dev)
        ii = sel[0][:, None, None]
        yy = (sel[1][:, None] + ar[None, :])[:, :, None]
        xx = (sel[2][:, None] + ar[None, :])[:, None, :]
        xb = U[ii, yy, xx]
        yb = L[ii, yy, xx]
        lr = 3e-3 if step < steps * 0.7 else 1e-3
        mf4d.mf4d_net_backward(th, xb, yb, g, 0.1, stats, ws)
        mf4d.mf4d_net_step(th, g, mm, vv, step, lr)
    torch.cuda.synchronize()
    train_s = time.time() - t1
    train_loss, train_acc = (float(v) for v in stats.cpu())
    del ws, U, L
    print(f"[bench] learned: {steps} steps x {B} crops in {train_s:.1f}s, loss {train_loss:.3f}, "
          f"last-batch accuracy {train_acc:.3f}", file=sys.stderr, flush=True)

    p = mf4d.Params(sig, mode=mf4d.MF4D_VALLEY, cycles=20, substeps=15)
    H = W = 2048
    ins = [torch.from_numpy(u).to(dev) for u in test_imgs]
    outs_p = [torch.empty_like(x) for x in ins]
    outs_l = [torch.empty_like(x) for x in ins]
    ws_p = mf4d.workspace(H, W, p, dev)
    ws_l = mf4d.learned_workspace(H, W, p, dev)
    fb = torch.zeros(1, dtype=torch.int32, device=dev)

    def plain():
        for x, y in zip(ins, outs_p):
            mf4d.mf4d_filter(x, y, p, ws_p)

    def learned(theta):
        for x, y in zip(ins, outs_l):
            mf4d.mf4d_filter_learned(x, y, p, theta, 0.9, fb, ws_l)

    plain()
    learned(th)
    ms_p = time_stream(torch, plain, reps)
    ms_l = time_stream(torch, lambda: learned(th), reps)
    ms_u = time_stream(torch, lambda: learned(th0), reps)
    # agreement with the exact sweep on the input images, and fallback share
    agree, agree_conf, conf_frac, fb_frac, fb_frac0 = [], [], [], 0.0, 0.0
    nws = mf4d.net_workspace(1, H, W, False, dev)
    for x, y in zip(ins, outs_l):
        exact = torch.empty((H, W), dtype=torch.uint8, device=dev)
        mf4d.mf4d_scale_select(x, p, exact, None, None, ws_p)
        pred = torch.empty_like(exact)
        conf = torch.empty((H, W), dtype=torch.float32, device=dev)
        mf4d.mf4d_net_forward(th, x, None, pred, conf, nws)
        ok = conf >= 0.9
        agree.append(float((pred == exact).float().mean()))
        agree_conf.append(float((pred[ok] == exact[ok]).float().mean()) if bool(ok.any()) else 1.0)
        conf_frac.append(float(ok.float().mean()))
        mf4d.mf4d_filter_learned(x, y, p, th, 0.9, fb, ws_l)
        torch.cuda.synchronize()
        fb_frac += int(fb.item()) / (20 * H * W) / len(ins)
        mf4d.mf4d_filter_learned(x, torch.empty_like(x), p, th0, 0.9, fb, ws_l)
        torch.cuda.synchronize()
        fb_frac0 += int(fb.item()) / (20 * H * W) / len(ins)
    d = torch.cat([(a.double() - b.double()).ravel() for a, b in zip(outs_l, outs_p)])
    ref = torch.cat([b.double().ravel() for b in outs_p])
    return {"images": len(ins), "size": [H, W], "cycles": 20, "substeps": 15, "scales": len(sig),
            "threshold": 0.9,
            "training": {"patches": steps * B, "patch_size": C, "batch": B, "steps": steps,
                         "pool": "64 images of 1024^2: 32 fundus type (seeds 10000-10031), 32 inverted ridge "
                                 "type (seeds 10032-10063); labels from the exact sweep",
                         "seconds": train_s, "loss_last_batch": train_loss, "accuracy_last_batch": train_acc},
            "plain_ms": ms_p, "learned_ms": ms_l, "untrained_learned_ms": ms_u,
            "plain_images_per_s": len(ins) / (ms_p * 1e-3), "learned_images_per_s": len(ins) / (ms_l * 1e-3),
            "untrained_learned_images_per_s": len(ins) / (ms_u * 1e-3),
            "speedup": ms_p / ms_l,
            "scale_agreement_cycle0": float(np.mean(agree)),
            "scale_agreement_confident_cycle0": float(np.mean(agree_conf)),
            "confident_fraction_cycle0": float(np.mean(conf_frac)),
            "fallback_fraction_all_cycles": fb_frac,
            "untrained_fallback_fraction_all_cycles": fb_frac0,
            "final_max_abs_vs_plain": float(d.abs().max()),
            "final_rel_l2_vs_plain": float(d.norm() / ref.norm())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="creases4096")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stages", action="store_true")
    ap.add_argument("--no-extensions", action="store_true", help="skip the extension comparisons (batched, learned, volume)")
    ap.add_argument("--eager", action="store_true", help="time eager mf4d_filter calls instead of graph replays")
    ap.add_argument("--only", choices=("batched", "learned", "volume", "aux"),
                    help="run only this extension comparison and print its JSON line (for profiling)")
    ap.add_argument("--learned-patches", type=int, default=20000, help="training crops of the learned comparison")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU decomposition is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1611_06906_amd import mf4d, synth

    if args.only:
        dev = torch.device("cuda:0")
        if args.only == "batched":
            res = batched_comparison(torch, mf4d, synth, dev)
        elif args.only == "learned":
            res = learned_comparison(torch, mf4d, synth, dev, patches=args.learned_patches)
        elif args.only == "aux":
            res = aux_comparison(torch, mf4d, synth, dev)
        else:
            res = volume_comparison(torch, mf4d, synth, dev)
        print(json.dumps({args.only: res}), flush=True)
        return

    w = synth.WORKLOADS[args.workload]()
    t0 = time.time()
    u_np = w.image()
    print(f"[bench] workload {w.name} {w.H}x{w.W} generated in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)
    dev = torch.device("cuda:0")
    p = mf4d.Params.from_workload(w)
    u_in = torch.from_numpy(u_np).to(dev)
    u_out = torch.empty_like(u_in)
    ws = mf4d.workspace(w.H, w.W, p, dev)
    torch.cuda.synchronize()

    eager = lambda: mf4d.mf4d_filter(u_in, u_out, p, ws)
    eager()   # the side streams of the concurrent scales exist before a capture
    torch.cuda.synchronize()
    step, launch = eager, "eager mf4d_filter calls"
    if not args.eager:
        # one whole filter call recorded into a hipGraph, replayed once per step
        try:
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                eager()
            step, launch = graph.replay, "hipGraph replays of one recorded mf4d_filter call"
        except RuntimeError as e:   # time the eager calls and say why
            torch.cuda.synchronize()
            launch = f"eager mf4d_filter calls (graph recording failed: {e})"
            print(f"[bench] {launch}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed region: K whole-filter steps (single rank: no barrier needed)
    ms = time_stream(torch, step, args.steps)
    px_sub = w.H * w.W * w.cycles * w.substeps
    value = px_sub / (ms * 1e-3) / 1e6
    print(f"[bench] {args.steps} steps ({launch}), {ms:.2f} ms/step, {value:.0f} Mpx-substeps/s", file=sys.stderr,
          flush=True)
    ms_eager = ms if step is eager else time_stream(torch, eager, args.steps)

    # roofline of the fused FED substep kernel as the filter launches it: same
    # kernel, shapes, substeps per launch and tensor planes of the workload
    n, taus = mf4d.mf4d_fed_plan(p)
    hrho = torch.empty((3, w.H, w.W), dtype=torch.float32, device=dev)
    dpar = torch.empty_like(hrho)
    idx = torch.empty((w.H, w.W), dtype=torch.uint8, device=dev)
    mf4d.mf4d_scale_select(u_in, p, idx, None, None, ws)
    mf4d.mf4d_tensor(u_in, idx, p, hrho, dpar, ws)
    uc = u_in.clone()
    ut = torch.empty_like(uc)
    spl = SUBSTEPS_PER_LAUNCH
    # k cycles' steps per call, k the least with k n a multiple of 2 spl: an
    # even number of full launches, so the timing holds only the substep
    # kernel (no remainder launch, no copy-back); k = 2 at n = 20
    import math
    kcyc = 2 * spl // math.gcd(n, 2 * spl)
    taus2 = np.concatenate([taus] * kcyc)
    launches = kcyc * n // spl
    assert (kcyc * n) % spl == 0 and launches % 2 == 0
    cyc = lambda: mf4d.mf4d_fed_cycle_tensor(uc, ut, dpar, taus2, spl)
    cyc()
    reps = 10
    ms_cycle = time_stream(torch, cyc, reps)
    us_launch = ms_cycle * 1e3 / launches
    t = us_launch * 1e-6
    m = w.H * w.W
    flops = SUBSTEP_FLOPS_PER_PX * spl * m / t
    hbm = SUBSTEP_BYTES_PER_PX * m / t
    traffic = counter_traffic(f"fed_stream2_kernel<{spl}>")
    roofline = {"bound": "hbm",
                "kernel": f"fed_stream2_kernel<{spl}> (fused FED substep, {spl} substeps per launch, two columns per lane)",
                "achieved": hbm / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": hbm / HBM_PEAK,
                "traffic": traffic,
                "traffic_unit": "B per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated)",
                "traffic_over_algorithmic": (traffic / (SUBSTEP_BYTES_PER_PX * m)) if traffic else None,
                "us_per_launch": us_launch, "bytes_per_px_launch": SUBSTEP_BYTES_PER_PX,
                "px_per_launch": m, "target_frac": 0.6, "meets_target": hbm / HBM_PEAK >= 0.6}
    # the same kernel's launches inside the filter (after each cycle's sweep)
    # run slower than back to back; their mean from the committed kernel trace
    in_filter = trace_mean_us(f"fed_stream2_kernel<{spl}>", f"fed_stream2_kernel<{spl}> [filter]")
    roofline["us_per_launch_in_filter"] = in_filter
    roofline["frac_in_filter"] = (SUBSTEP_BYTES_PER_PX * m / (in_filter * 1e-6) / HBM_PEAK) if in_filter else None
    roofline_alu = {"bound": "alu", "kernel": roofline["kernel"], "achieved": flops / 1e12,
                    "peak": VALU_PEAK / 1e12, "unit": "TFLOP/s", "frac": flops / VALU_PEAK,
                    "flops_per_px_substep": SUBSTEP_FLOPS_PER_PX, "us_per_launch": us_launch,
                    "peak_note": "FP32 vector without packed FP32: 256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz"}
    # the same kernel at one substep per launch is HBM-bound: report it too
    ms1 = time_stream(torch, lambda: mf4d.mf4d_fed_cycle_tensor(uc, ut, dpar, taus2, 1), reps)
    t1 = ms1 * 1e-3 / (kcyc * n)
    roofline_single = {"bound": "hbm", "kernel": "fed_stream_kernel<1> (one column per lane)", "achieved": SUBSTEP_BYTES_PER_PX * m / t1 / 1e9,
                       "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": SUBSTEP_BYTES_PER_PX * m / t1 / HBM_PEAK,
                       "us_per_launch": t1 * 1e6}

    # the fused sweep kernel at the largest scale, sigma = 16 (radius 48, 8
    # chunks of 16 inputs): a one-scale selection is that kernel plus a
    # per-pixel argmax over one scale (S, blob read; index written), so the
    # rate below is a lower bound on the kernel's own
    p16 = mf4d.Params([16.0], mode=w.mode, lam=w.lam, rho=w.rho, beta=w.beta)
    sel16 = lambda: mf4d.mf4d_scale_select(u_in, p16, idx, None, None, ws)
    sel16()
    t16 = time_stream(torch, sel16, reps) * 1e-3
    R16 = 49                                  # ceil(3 sigma) + 1: support of the difference taps
    sweep_flops_px = 8 * (2 * R16 + 1) * 2    # 3 horizontal + 5 vertical filters
    # the banded Toeplitz products as issued: 8 chunks of 16 inputs taken as
    # 4 slices of 32, each FP32 product as 6 BF16 part products
    nc16 = (16 + 2 * R16 + 15) // 16
    bf16_flops_px = 8 * (16 * nc16) * BF3_PRODUCTS * 2
    peak_eq = MFMA_BF16_PEAK / BF3_PRODUCTS
    achieved = sweep_flops_px * m / t16
    roofline_sweep = {"bound": "mfma", "kernel": "sweep_fused_kernel<8> (both passes of sigma = 16, split-BF16 "
                                                 "products) + one-scale argmax",
                      "achieved": achieved / 1e12, "peak": peak_eq / 1e12, "unit": "TFLOP/s",
                      "frac": achieved / peak_eq,
                      "peak_note": "FP32-equivalent: dense BF16 peak / 6 part products",
                      "traffic": counter_traffic("sweep_fused_kernel<8>", "sweep_fused_kernel<8> [select]"),
                      "us_per_launch": t16 * 1e6, "flops_per_px": sweep_flops_px,
                      "bf16_issued_TFLOPs": bf16_flops_px * m / t16 / 1e12,
                      "bf16_issued_frac": bf16_flops_px * m / t16 / MFMA_BF16_PEAK,
                      "fp32_mfma_peak_frac": achieved / MFMA_F32_PEAK,
                      # a selection does not form N: u read 4, S and blob written 8
                      "hbm_bytes_per_px": 12, "hbm_achieved_GBs": 12 * m / t16 / 1e9}

    # a one-substep cycle from H_rho: that substep plus the plain copy of H*W
    # floats back into u (4 B read + 4 B write per pixel), the reference for
    # HBM counters
    mf4d.mf4d_fed_cycle(uc, ut, hrho, p, taus[:1])
    torch.cuda.synchronize()

    # a plain device copy of 1 GiB (torch's copy kernel): the HBM rate this
    # box reaches in practice, against which the rooflines can be read
    csrc_ = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    cdst = torch.empty_like(csrc_)
    cdst.copy_(csrc_)
    ms_copy = time_stream(torch, lambda: cdst.copy_(csrc_), 5)
    copy_bytes = 2 * csrc_.numel() * 4
    hbm_copy_probe = {"kernel": "torch copy_ of 1 GiB float32 (read + write)", "bytes": copy_bytes, "ms": ms_copy,
                      "GB/s": copy_bytes / (ms_copy * 1e-3) / 1e9,
                      "frac_of_peak": copy_bytes / (ms_copy * 1e-3) / HBM_PEAK}
    del csrc_, cdst

    stages = None
    if not args.no_stages:
        sel_ms = time_stream(torch, lambda: mf4d.mf4d_scale_select(u_in, p, idx, None, None, ws), 3)
        ten_ms = time_stream(torch, lambda: mf4d.mf4d_tensor(u_in, idx, p, hrho, dpar, ws), 3)
        stages = {"per_cycle_scale_select_ms": sel_ms, "per_cycle_tensor_incl_sweep_ms": ten_ms,
                  "per_cycle_substeps_ms": ms_cycle / 2, "cycles": w.cycles}

    # rows a2-a4 per cycle: the filter's time outside its substep launches
    launches_per_cycle = (w.substeps + spl - 1) // spl
    sel_cycle_ms = ms / w.cycles - launches_per_cycle * us_launch * 1e-3
    sel_bytes = SELECTION_BYTES_PER_PX * m
    sel_traffic = selection_traffic()
    roofline_selection = {"bound": "hbm", "stages": "scale sweep (8 scales) + argmax + integration, per cycle",
                          "achieved": sel_bytes / (sel_cycle_ms * 1e-3) / 1e9, "peak": HBM_PEAK / 1e9,
                          "unit": "GB/s", "frac": sel_bytes / (sel_cycle_ms * 1e-3) / HBM_PEAK,
                          "ms_per_cycle": sel_cycle_ms, "bytes_per_px": SELECTION_BYTES_PER_PX,
                          "traffic": sel_traffic, "traffic_unit": "B per cycle (copy-calibrated counters)",
                          "traffic_over_algorithmic": (sel_traffic / sel_bytes) if sel_traffic else None}

    extensions = None
    if not args.no_extensions:
        extensions = {"batched_256": batched_comparison(torch, mf4d, synth, dev)}
        print(f"[bench] batched: {json.dumps(extensions['batched_256'])}", file=sys.stderr, flush=True)
        extensions["learned_2048"] = learned_comparison(torch, mf4d, synth, dev, patches=args.learned_patches)
        print(f"[bench] learned: {json.dumps(extensions['learned_2048'])}", file=sys.stderr, flush=True)
        extensions["volume_256"] = volume_comparison(torch, mf4d, synth, dev)
        print(f"[bench] volume: {json.dumps(extensions['volume_256'])}", file=sys.stderr, flush=True)
        extensions["aux_4096"] = aux_comparison(torch, mf4d, synth, dev)
        print(f"[bench] aux: {json.dumps(extensions['aux_4096'])}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        cores = len(os.sched_getaffinity(0))
        omp = int(os.environ.get("OMP_NUM_THREADS", cores))
        t1 = time.time()
        oracle.filter(u_np, w.sigmas, w.mode, lam=w.lam, rho=w.rho, beta=w.beta, cycles=CPU_CYCLES,
                      substeps=w.substeps, tau_max=w.tau_max)
        dt = time.time() - t1
        cpu = {"value": w.H * w.W * w.substeps * CPU_CYCLES / dt / 1e6, "unit": "Mpixel-FED-substeps/s",
               "cores": min(omp, cores), "kind": "oracle",
               "sample": f"the first {CPU_CYCLES} of {w.cycles} cycles ({w.substeps} substeps each) of the full "
                         f"{w.H}x{w.W} image, FP64, {dt:.1f} s"}

    out = {
        "metric": "Mpixel-FED-substeps/s and % HBM roofline, plain vs batched/learned @ oracle tol",
        "value": value,
        "unit": "Mpixel-FED-substeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "ms_per_step_eager": ms_eager,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.H}x{w.W} creases, {len(w.sigmas)} scales 1-16, "
                               f"ridge+valley, {w.cycles} FED cycles x {w.substeps} substeps, plain path",
                   "H": w.H, "W": w.W, "cycles": w.cycles, "substeps": w.substeps,
                   "nscales": len(w.sigmas), "mode": "both", "path": "plain", "launch": launch},
        "roofline": roofline,
        "roofline_alu": roofline_alu,
        "roofline_selection": roofline_selection,
        "roofline_single_substep": roofline_single,
        "roofline_sweep": roofline_sweep,
        "hbm_copy_probe": hbm_copy_probe,
        "cpu_baseline": cpu,
        "stages": stages,
        "extensions": extensions,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
