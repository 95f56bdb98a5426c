"""Benchmark: direct incoherent dedispersion of one survey-shaped beam on one GPU.

Workload (one "step" = one whole transform of one beam, the full hot path):
2-bit packed time-major filterbank, 1024 channels, 2^19 samples of 64 us
(33.6 s), f_top 1581.8 MHz, df -0.390625 MHz, 1024 trial DMs in [0, 1000)
pc cm^-3, uint32 output [1024][2^19 - 20456].  Seeded synthetic levels with
8 injected pulses.  The input is resident in HBM before timing starts.

Prints one JSON line.  `value` is dedispersed outputs (DM x sample) per second
over the timed steps; the dominant kernel's duration is measured per launch
with HIP events on the stream it runs on.  The CPU oracle is timed on a
bounded DM subset of the same beam (`cpu_baseline`).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X peaks used for the roofline.  VALU: 256 CUs x 4 SIMDs x 16 lanes x
# 2.4 GHz = 39.32 T 32-bit lane operations/s (a wave64 instruction occupies a
# SIMD for 4 cycles).  The sums are exact integer adds in packed lanes
# (Section 2.3, bit-level parallelism): a 32-bit lane operation can add at
# most eight 2-bit codes (4-bit lanes) or two 8-bit codes (16-bit lanes), so
# the ALU roofline in channel-adds/s is 8x (2-bit) or 2x (8-bit) the lane-op
# rate.  HBM3E: 8 TB/s.
VALU_LANE_OPS_PER_S = 256 * 4 * 16 * 2.4e9
SIMDS = 256 * 4
XCDS = 8
ADDS_PER_LANE_OP = {2: 8, 8: 2}
HBM_PEAK_GBS = 8000.0
# the sources the tiled kernel is compiled from (their digest keys the
# committed counters to the code they were taken on)
KERNEL_SOURCES = ("dedisp_kernels.hip", "dedisp_device.h")


def alu_peak_tadds(nbits):
    return ADDS_PER_LANE_OP[nbits] * VALU_LANE_OPS_PER_S / 1e12


def kernel_source_sha():
    import hashlib
    csrc = os.path.join(ROOT, "paper_1201_5380_amd", "csrc")
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()


def tile_arg(text):
    """A tile shape from "waves,dms_per_wave,words_per_lane,chunk_chans[,sample_format]"."""
    v = [int(x) for x in text.split(",")]
    if len(v) not in (4, 5):
        raise ValueError(f"tile shape {text!r}: four or five integers")
    return dict(kind=0, waves=v[0], dms_per_wave=v[1], words_per_lane=v[2], chunk_chans=v[3],
                sample_format=v[4] if len(v) == 5 else -1)


def counters_for(path, workload, tile):
    """The committed rocprofv3 counter entry for this workload and tile shape,
    if it was taken on the current kernel sources (else None)."""
    try:
        entries = json.load(open(path)).get("entries", [])
    except (OSError, ValueError):
        return None
    sha = kernel_source_sha()
    for e in entries:
        if e.get("workload") == workload and e.get("tile") == tile and e.get("kernel_source_sha256") == sha:
            return e
    return None


def roofline_block(nbits, adds, kernel_ms, ctr):
    """Roofline of the dominant kernel: achieved channel-adds/s against the ALU
    peak of the lanes the adds run in; HBM bytes and VALU issue from counters."""
    achieved = adds / (kernel_ms * 1e-3) / 1e12
    peak = alu_peak_tadds(nbits)
    blk = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tadd/s",
           "frac": achieved / peak, "traffic": None, "valu_issue": None, "lds_busy": None,
           "counters_kernel_us": None}
    if ctr:
        blk["traffic"] = ctr.get("hbm_bytes_per_launch")
        cyc = ctr.get("grbm_gui_active")             # summed over the XCDs
        if cyc:
            per_xcd = cyc / XCDS
            blk["valu_issue"] = ctr["sq_insts_valu"] * 4 / (SIMDS * per_xcd)
            if ctr.get("sq_lds_idx_active"):
                blk["lds_busy"] = ctr["sq_lds_idx_active"] / (per_xcd * 256)   # per CU cycle
            blk["counters_kernel_us"] = per_xcd / 2.4e3
        blk["counters_kernel"] = ctr.get("kernel")
    return blk


def _counter_rows(d):
    """(kernel name, dispatch id, counter, value) rows of every rocprofv3
    counter-collection CSV under directory d."""
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                rows.append((r.get("Kernel_Name", ""), (f, r.get("Dispatch_Id")), r["Counter_Name"],
                             float(r["Counter_Value"])))
    return rows


def _per_dispatch_means(d, pick):
    """Mean per dispatch of every counter over the dispatches of the kernel
    `pick` selects (summed over the rows of one dispatch, e.g. per XCD)."""
    per = {}
    names = {}
    for name, disp, ctr, val in _counter_rows(d):
        if not pick(name):
            continue
        names[disp] = name
        per.setdefault(ctr, {}).setdefault(disp, 0.0)
        per[ctr][disp] += val
    means = {c: sum(v.values()) / len(v) for c, v in per.items()}
    kernels = sorted(set(names.values()))
    return means, kernels, len(names)


def summarize_counters(args):
    """Fold rocprofv3 --pmc passes of the dominant kernel into the counters
    file the roofline reads (one entry per workload, tile and kernel source
    digest), with HBM bytes scaled by what the same counters read for a
    plain 1 GiB device copy."""
    w, dpw, m, cc, fmt = (int(x) for x in args.tile_key.split(","))
    tile = dict(kind=0, waves=w, dms_per_wave=dpw, words_per_lane=m, chunk_chans=cc, sample_format=fmt)
    sub = args.kernel_filter
    means, kernels = {}, set()
    for d in args.summarize_counters:
        mm, ks, nd = _per_dispatch_means(d, lambda n: sub in n)
        means.update(mm)
        kernels.update(ks)
    def copy_pick(n):
        return "copy" in n.lower()
    cf, _, _ = _per_dispatch_means(args.calibration_dirs[0], copy_pick)
    cw, _, _ = _per_dispatch_means(args.calibration_dirs[1], copy_pick)
    gib = float(1 << 30)
    fs = gib / (cf["FETCH_SIZE"] * 1024.0)
    ws = gib / (cw["WRITE_SIZE"] * 1024.0)
    entry = {"workload": args.workload, "tile": tile, "kernel": sorted(kernels),
             "kernel_source_sha256": kernel_source_sha(), "counters_per_dispatch": means,
             "fetch_scale_from_copy": fs, "write_scale_from_copy": ws}
    if "FETCH_SIZE" in means and "WRITE_SIZE" in means:
        entry["hbm_bytes_per_launch"] = (means["FETCH_SIZE"] * fs + means["WRITE_SIZE"] * ws) * 1024.0
    for key, ctr in (("grbm_gui_active", "GRBM_GUI_ACTIVE"), ("sq_insts_valu", "SQ_INSTS_VALU"),
                     ("sq_lds_idx_active", "SQ_LDS_IDX_ACTIVE")):
        if ctr in means:
            entry[key] = means[ctr]
    try:
        doc = json.load(open(args.counters_json))
    except (OSError, ValueError):
        doc = {"entries": []}
    doc["entries"] = [e for e in doc.get("entries", [])
                      if not (e.get("workload") == args.workload and e.get("tile") == tile)] + [entry]
    with open(args.counters_json, "w") as fh:
        json.dump(doc, fh, indent=1, sort_keys=True)
    print(json.dumps(entry, indent=1, sort_keys=True))


def host_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "host_cpus": os.cpu_count()}


def gpu_info(torch):
    prop = torch.cuda.get_device_properties(0)
    info = {"name": prop.name, "arch": getattr(prop, "gcnArchName", None),
            "compute_units": prop.multi_processor_count, "sclk_mhz": None}
    # current shader clock from the driver's DPM table, where readable
    import glob
    for f in glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk"):
        try:
            for line in open(f):
                if line.strip().endswith("*"):
                    info["sclk_mhz"] = line.split(":")[1].strip().rstrip("*").strip()
        except OSError:
            continue
        if info["sclk_mhz"]:
            break
    return info


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # the paper's protocol (Section 5.2): repeated runs, median and 5th/95th percentiles
    ap.add_argument("--steps", type=int, default=101)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--nsamps", type=int, default=1 << 19)
    ap.add_argument("--no-tune", action="store_true", help="use the default tile shape")
    ap.add_argument("--tile", default=None,
                    help="waves,dms_per_wave,words_per_lane,chunk_chans[,sample_format]: use this shape, "
                         "no tuning")
    ap.add_argument("--tune-cache", default=None)
    ap.add_argument("--large-tile", default=None,
                    help="waves,dms_per_wave,words_per_lane,chunk_chans[,sample_format] for the large beam: "
                         "no tuning")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate CPU time budget for the oracle baseline")
    ap.add_argument("--counters-json", default=os.path.join(ROOT, "profiles", "counters.json"),
                    help="rocprofv3 counters per launch (HBM bytes, VALU instructions), if present")
    ap.add_argument("--summarize-counters", nargs="+", default=None, metavar="DIR",
                    help="fold rocprofv3 --pmc output directories of one kernel into --counters-json "
                         "and exit (needs --workload, --tile-key, --calibration-dirs)")
    ap.add_argument("--workload", default=None)
    ap.add_argument("--tile-key", default=None, help="waves,dms_per_wave,words_per_lane,chunk_chans,format")
    ap.add_argument("--kernel-filter", default="k_tiled")
    ap.add_argument("--calibration-dirs", nargs=2, default=None, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="rocprofv3 FETCH_SIZE and WRITE_SIZE passes over --calibrate-copy")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--no-systems", action="store_true",
                    help="skip the batched and serving measurements")
    ap.add_argument("--serve-seconds", type=float, default=12.0)
    ap.add_argument("--legs", default="scrunched,subband,tree,large_beam,tiny,batched,serving",
                    help="comma-separated systems legs to run after the headline transform")
    return ap.parse_args()


def bench_batch(torch, dev, steps):
    """The 13-beam batched workload: one graph launch vs the beams run one by one."""
    from paper_1201_5380_amd import Batch, Plan, synth
    beams, plain_ms, outputs, adds = [], [], 0, 0
    for b in range(13):
        prm = synth.batch_beam_params(b)
        plan = Plan(prm["nchans"], prm["dt"], prm["f_top"], prm["df"], prm["nbits"]).set_dm_list(
            synth.dm_list_linear(prm["ndm"], prm["dm_max"]))
        n = prm["nsamps"]
        inp = torch.from_numpy(synth.batch_beam(b).packed().reshape(-1)).to(dev)
        out = torch.empty((plan.ndm, n - plan.max_delay), dtype=torch.int32, device=dev)
        beams.append((plan, inp, n, out, 0))
        outputs += plan.ndm * (n - plan.max_delay)
        adds += plan.ndm * (n - plan.max_delay) * prm["nchans"]
    # plain form: each beam alone with its own tuned shape
    for plan, inp, n, out, _ in beams:
        plan.tune(inp, out, n)
        for _ in range(2):
            plan.execute(inp, n, out=out)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            plan.execute(inp, n, out=out)
        e1.record()
        torch.cuda.synchronize()
        plain_ms.append(e0.elapsed_time(e1) / steps)
    batch = Batch(beams)
    for _ in range(2):
        batch.execute()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        batch.execute()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    return {"workload": "13 beams: nchans 1024 (8-bit) / 512 (2-bit), Nt in [2^16, 2^19], "
                        "256-1024 DMs up to DM_max in [300, 1500]",
            "graph_ms": ms, "outputs_per_s": outputs / (ms * 1e-3),
            "channel_adds_per_s": adds / (ms * 1e-3),
            "plain_sum_ms": float(sum(plain_ms)),
            "plain_ms_per_beam": [round(x, 3) for x in plain_ms],
            "plain_tiles": [p.tile_config() for p, *_ in beams],
            "plain_outputs_per_s": outputs / (sum(plain_ms) * 1e-3),
            "batched_over_plain": float(sum(plain_ms)) / ms}


def bench_scrunched(torch, dev, plan, inp, nsamps, steps, direct_ms):
    """The survey beam with time-scrunching (Section 2.1): default factors up
    to 64, each factor group tuned; the same input as the direct transform."""
    factors = plan.default_scrunch_factors(64)
    plan.set_scrunching(factors)
    lens = plan.output_lengths(nsamps)
    out = torch.empty((plan.ndm, int(lens.max())), dtype=torch.int32, device=dev)
    tune_ms = plan.tune(inp, out, nsamps)
    for _ in range(2):
        plan.execute(inp, nsamps, out=out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        plan.execute(inp, nsamps, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    plan.set_scrunching(None)
    groups = {int(f): int((factors == f).sum()) for f in sorted(set(factors.tolist()))}
    return {"workload": "survey beam, default scrunch factors (1 up to the diagonal DM, doubling "
                        "at each power-of-two multiple of it, at most 64)",
            "diagonal_dm": plan.diagonal_dm(), "trials_per_factor": groups,
            "ms": ms, "tune_ms": tune_ms, "outputs": int(lens.sum()),
            "outputs_per_s": float(lens.sum()) / (ms * 1e-3),
            "speedup_vs_direct": direct_ms / ms}


def bench_subband(torch, dev, plan, inp, nsamps, steps, direct_ms, nsub=32, ngroup=32,
                  sweep=((16, 16), (64, 32), (64, 64))):
    """The survey beam with sub-band dedispersion (Section 4): 32-channel
    sub-bands, 32 trials per nominal DM (the balanced choice N'_DM = N'_nu),
    each pass tuned; the same input as the direct transform.  `sweep` times
    other (sub-band width, trials per nominal DM) pairs: wider sub-bands and
    more trials per nominal DM do less work and smear more (Appendix B)."""
    def timed(ns, ng):
        plan.set_subband(ns, ng)
        nout = int(plan.output_lengths(nsamps)[0])
        out = torch.empty((plan.ndm, nout), dtype=torch.int32, device=dev)
        tune_ms = plan.tune(inp, out, nsamps)
        for _ in range(2):
            plan.execute(inp, nsamps, out=out)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            plan.execute(inp, nsamps, out=out)
        e1.record()
        torch.cuda.synchronize()
        plan.set_subband(0, 0)
        del out
        return e0.elapsed_time(e1) / steps, tune_ms, nout

    ms, tune_ms, nout = timed(nsub, ngroup)
    res = {"workload": f"survey beam, sub-bands of {nsub} channels, {ngroup} trials per nominal DM",
           "ms": ms, "tune_ms": tune_ms, "nout": nout,
           "outputs_per_s": plan.ndm * nout / (ms * 1e-3),
           "speedup_vs_direct": direct_ms / ms, "sweep": []}
    for ns, ng in sweep:
        m, _, n = timed(ns, ng)
        res["sweep"].append({"nsub": ns, "trials_per_nominal_dm": ng, "ms": m,
                             "speedup_vs_direct": direct_ms / m})
    return res


def bench_tree(torch, dev, beam, inp, nsamps, steps, nsub=32):
    """The survey beam through the piecewise linear tree (Section 3) with
    32-channel sub-bands, against the direct transform of the same trials:
    the survey's own trials up to the tree's diagonal DM, a dense list of
    1024 trials spread evenly below it (the regime the tree is built for),
    4096 trials up to 4x the diagonal (four stage-1 passes) and all of the
    survey's trials (up to ~31x the diagonal)."""
    import numpy as np
    from paper_1201_5380_amd import Plan
    k = 4.148808e3 / beam.dt
    fb = beam.f_top + beam.nchans * beam.df
    fa = beam.f_top + (beam.nchans - nsub) * beam.df
    diag = (nsub - 0.5) / (k * (1 / fb ** 2 - 1 / beam.f_top ** 2) - k * (1 / fa ** 2 - 1 / beam.f_top ** 2))

    def timed(plan):
        nout = int(plan.output_lengths(nsamps).max())
        out = torch.empty((plan.ndm, nout), dtype=torch.int32, device=dev)
        plan.tune(inp, out, nsamps)
        for _ in range(2):
            plan.execute(inp, nsamps, out=out)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            plan.execute(inp, nsamps, out=out)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps, nout

    res = {}
    for key, dms, what in (("survey_trials", beam.dms[beam.dms < diag], "the survey's trials"),
                           ("dense_trials", np.linspace(0.0, 0.999 * diag, 1024), "1024 evenly spaced trials"),
                           ("dense_beyond", np.linspace(0.0, 4.0 * diag, 4096, endpoint=False),
                            "4096 evenly spaced trials (4 passes)"),
                           ("survey_all", beam.dms, "all of the survey's trials (31 passes)")):
        direct = Plan(beam.nchans, beam.dt, beam.f_top, beam.df, beam.nbits).set_dm_list(dms)
        d_ms, _ = timed(direct)
        tree = Plan(beam.nchans, beam.dt, beam.f_top, beam.df, beam.nbits).set_dm_list(dms).set_tree(nsub)
        t_ms, nout = timed(tree)
        if key == "survey_all":
            # the paper's procedure for large DMs: scrunch, then the tree at
            # each factor (default factors up to 64), beside the scrunched
            # direct transform with the same factors
            f = direct.default_scrunch_factors(64)
            direct.set_scrunching(f)
            ds_ms, _ = timed(direct)
            tree.set_tree(0).set_scrunching(f).set_tree(nsub)
            ts_ms, _ = timed(tree)
            outs = int(tree.output_lengths(nsamps).sum())
            res["survey_all_scrunched"] = {
                "workload": f"survey beam, all of the survey's trials ({len(dms)}) up to DM "
                            f"{float(dms.max()):.2f}, default scrunch factors up to 64, then the tree with "
                            f"sub-bands of {nsub} channels at each factor",
                "ms": ts_ms, "outputs": outs, "outputs_per_s": outs / (ts_ms * 1e-3),
                "direct_scrunched_ms_same_factors": ds_ms, "direct_ms_unscrunched": d_ms,
                "speedup_vs_direct_scrunched": ds_ms / ts_ms, "speedup_vs_direct": d_ms / ts_ms}
        res[key] = {"workload": f"survey beam, {what} ({len(dms)}) up to DM {float(dms.max()):.2f} "
                                f"(piecewise diagonal {diag:.2f}), sub-bands of {nsub} channels",
                    "ms": t_ms, "nout": nout, "outputs_per_s": len(dms) * nout / (t_ms * 1e-3),
                    "direct_ms_same_trials": d_ms, "speedup_vs_direct": d_ms / t_ms}
    return res


def copy_times(torch, dev, packed, out, ms_per_step):
    """Host-to-device copy of the survey input and device-to-host copy of its
    outputs, from and to pinned host memory (the transform itself takes its
    input already in HBM), and the outputs/s a caller handing over host
    buffers would see with copies and transform in sequence."""
    host_in = torch.from_numpy(packed.reshape(-1)).pin_memory()
    dev_in = torch.empty_like(host_in, device=dev)
    host_out = torch.empty(out.shape, dtype=out.dtype).pin_memory()

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    h2d = timed(lambda: dev_in.copy_(host_in, non_blocking=True))
    d2h = timed(lambda: host_out.copy_(out, non_blocking=True))
    n_in, n_out = host_in.numel(), out.numel() * 4
    return {"h2d_ms": h2d, "h2d_GBs": n_in / (h2d * 1e-3) / 1e9, "d2h_ms": d2h,
            "d2h_GBs": n_out / (d2h * 1e-3) / 1e9,
            "pcie_inclusive_outputs_per_s": out.numel() / ((h2d + ms_per_step + d2h) * 1e-3)}


def bench_tiny(torch, dev, reps=200):
    """The tiny 8-bit case: 4096 samples x 64 channels of 64 us, f_top 1500 MHz,
    df -1 MHz, 32 DMs in [0, 100) (launch-bound; a parity case, reported but
    not the roofline's workload)."""
    from paper_1201_5380_amd import Plan, synth
    b = synth.tiny_beam()
    plan = Plan(b.nchans, b.dt, b.f_top, b.df, b.nbits).set_dm_list(b.dms)
    b.inject(lambda i: plan.delay_table()[i])
    nsamps = b.nsamps
    inp = torch.from_numpy(np.ascontiguousarray(b.packed()).reshape(-1)).to(dev)
    nout = nsamps - plan.max_delay
    out = torch.empty((plan.ndm, nout), dtype=torch.int32, device=dev)
    plan.tune(inp, out, nsamps)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for _ in range(5):
        plan.execute(inp, nsamps, out=out)
    torch.cuda.synchronize()
    for e0, e1 in ev:
        e0.record()
        plan.execute(inp, nsamps, out=out)
        e1.record()
    torch.cuda.synchronize()
    ms = np.array([e0.elapsed_time(e1) for e0, e1 in ev])
    return {"workload": "tiny beam: 8-bit, 64 ch, 4096 samples x 64 us, 32 DMs in [0, 100), "
                        "f_top 1500 MHz, df -1 MHz",
            "median_ms": float(np.median(ms)), "p95_ms": float(np.percentile(ms, 95)),
            "outputs_per_s": plan.ndm * nout / (float(np.median(ms)) * 1e-3), "tile": plan.tile_config()}


def bench_large(torch, dev, steps, counters_json, tile=None, cache_path=None):
    """The large 8-bit beam: 2^20 samples x 4096 channels of 54.6 us,
    f_top 1500 MHz, df -0.09765625 MHz, 2048 DMs in [0, 2000); seeded
    rint(N(128, 20)) noise clipped to [0, 255] made on the host."""
    from paper_1201_5380_amd import Plan, synth
    t0 = time.perf_counter()
    b = synth.large_beam()
    packed = b.packed()
    sha = synth.sha256(packed)
    gen_s = time.perf_counter() - t0
    nsamps, nchans, ndm = b.nsamps, b.nchans, len(b.dms)
    plan = Plan(nchans, b.dt, b.f_top, b.df, 8).set_dm_list(b.dms)
    inp = torch.from_numpy(packed.reshape(-1)).to(dev)
    del b, packed
    nout = nsamps - plan.max_delay
    out = torch.empty((ndm, nout), dtype=torch.int32, device=dev)
    if tile:
        plan.set_tile_config(tile_arg(tile))
    else:
        plan.tune(inp, out, nsamps, cache_path=cache_path)
    plan.execute(inp, nsamps, out=out)
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    for e0, e1 in ev:
        e0.record(stream)
        plan.execute(inp, nsamps, out=out, stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    ms = np.array([e0.elapsed_time(e1) for e0, e1 in ev])
    med = float(np.median(ms))
    adds = ndm * nout * nchans
    cfg = plan.tile_config()
    return {"workload": "large beam: 8-bit, 4096 ch, 1048576 samples x 54.6 us, 2048 DMs in [0, 2000), "
                        "f_top 1500 MHz, df -0.09765625 MHz",
            "ms": med, "ms_p5": float(np.percentile(ms, 5)), "ms_p95": float(np.percentile(ms, 95)),
            "runs": steps, "nout": nout, "outputs_per_s": ndm * nout / (med * 1e-3),
            "channel_adds_per_s": adds / (med * 1e-3),
            "roofline": roofline_block(8, adds, med, counters_for(counters_json, "large-8bit-4096ch", cfg)),
            "input_sha256": sha, "input_gen_s": gen_s, "tile": cfg}


def bench_serve(torch, dev, seconds):
    """32 streams, chunks of U[2^14, 2^18] samples arriving as a Poisson process at
    4x real time per stream (aggregate ~14.4 chunks/s), 64 GB admission budget."""
    from paper_1201_5380_amd import Plan, synth
    from paper_1201_5380_amd.serve import GpuExecutor, Server
    nstreams, nchans = 32, 1024
    plan = Plan(nchans, 64e-6, 1581.8, -0.390625, 2).set_dm_list(synth.dm_list_linear(1024, 1000.0))
    rb = plan.row_bytes
    pool_rows = (1 << 19) + (1 << 18)
    pool = torch.from_numpy(synth.pack(synth.stream_codes(0, pool_rows, nchans), 2)).pin_memory()
    pool_np = pool.numpy().reshape(pool_rows, rb)
    mean_len = ((1 << 14) + (1 << 18)) / 2
    rate = nstreams * 4.0 / (mean_len * 64e-6)
    narr = int(rate * seconds) + 1
    t_arr, sids = synth.poisson_arrivals(narr, rate, nstreams, seed=5)
    lens = {s: list(synth.stream_chunk_lengths(s, narr)) for s in range(nstreams)}
    offs = [(s * 104729) % (1 << 19) for s in range(nstreams)]

    def chunk_of(s):
        L = int(lens[s].pop(0))
        o = offs[s]
        offs[s] = (o + L) % (1 << 19)
        return pool_np[o:o + L]

    def consume(r):
        # the consumer takes the result and lets its device memory go
        r.out = None

    def run(open_loop):
        ex = GpuExecutor([plan] * nstreams, device=dev, max_chunk=1 << 18)
        ex.tune(1 << 18)
        srv = Server(ex, nstreams, budget_bytes=64 << 30, max_tick=16, max_inflight_ticks=4,
                     on_done=consume).start()
        reqs = []
        t0 = time.perf_counter()
        for ta, s in zip(t_arr, sids):
            if open_loop:
                delay = t0 + ta - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
            reqs.append(srv.submit(int(s), chunk_of(int(s))))
        srv.drain()
        wall = time.perf_counter() - t0
        srv.stop()
        st = srv.stats()
        outs = sum(r.n_out for r in reqs) * plan.ndm
        rt = np.array([r.nsamps * 64e-6 for r in reqs])
        lat = np.array([r.latency for r in reqs])
        st.update({"wall_s": wall, "outputs_per_s": outs / wall,
                   "p99_latency_over_chunk_duration": float(np.percentile(lat / rt, 99))})
        return st

    open_loop = run(True)
    offs[:] = [(s * 7919) % (1 << 19) for s in range(nstreams)]
    lens.update({s: list(synth.stream_chunk_lengths(s, narr)) for s in range(nstreams)})
    chunk_lens = [int(lens[int(s)][k]) for s, k in zip(sids, _per_stream_index(sids))]
    saturated = run(False)
    saturated["plain_same_chunks_outputs_per_s"] = plain_same_chunks(torch, dev, plan, chunk_lens)
    return {"workload": "32 streams x 2-bit 1024 ch, 1024 DMs in [0, 1000); chunks U[2^14, 2^18] "
                        f"samples, Poisson arrivals at {rate:.1f} chunks/s (4x real time per stream), "
                        "64 GB budget",
            "open_loop": open_loop, "saturated": saturated}


def _per_stream_index(sids):
    """(stream, k) -> k-th chunk of that stream, in arrival order, as stream ids."""
    seen = {}
    out = []
    for s in sids:
        k = seen.get(int(s), 0)
        seen[int(s)] = k + 1
        out.append(k)
    return out


def plain_same_chunks(torch, dev, plan, chunk_lens):
    """The plain transform over the serving run's chunk lengths, one execute
    per chunk of L new samples plus max_delay history samples already in HBM,
    back to back on one stream: the plain form's rate on the serving work."""
    nmax = max(chunk_lens) + plan.max_delay
    inp = torch.zeros(nmax * plan.row_bytes, dtype=torch.uint8, device=dev)
    out = torch.empty((plan.ndm, max(chunk_lens)), dtype=torch.int32, device=dev)
    plan.tune(inp, out, nmax)
    for L in chunk_lens[:4]:
        plan.execute(inp, L + plan.max_delay, out=out, out_row_stride=max(chunk_lens))
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for L in chunk_lens:
        plan.execute(inp, L + plan.max_delay, out=out, out_row_stride=max(chunk_lens))
    e1.record()
    torch.cuda.synchronize()
    return sum(chunk_lens) * plan.ndm / (e0.elapsed_time(e1) * 1e-3)


def cpu_baseline(packed, nsamps, nchans, nbits, table, budget_s):
    """Time the oracle on the first k DM rows of the beam (whole time range)."""
    import oracle
    ndm = table.shape[0]
    nout = nsamps - int(table.max())
    mx = int(table.max())
    # calibrate on one DM row per thread, then size the sample to the budget
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    oracle.dedisperse(packed, nsamps, nchans, nbits, table[:threads], max_delay=mx)
    per_round = time.perf_counter() - t0
    rounds = max(1, int(budget_s / max(per_round, 1e-6)))
    k = max(1, min(ndm, rounds * threads))
    t0 = time.perf_counter()
    oracle.dedisperse(packed, nsamps, nchans, nbits, table[:k], max_delay=mx)
    dt = time.perf_counter() - t0
    return {"value": k * nout / dt, "unit": "outputs/s", "cores": threads, "kind": "oracle",
            "cpu_model": host_info()["cpu_model"],
            "sample": f"first {k} of {ndm} DM rows x all {nout} output samples "
                      f"({k * nout * nchans:.3g} channel-adds) in {dt:.2f} s",
            "adds_per_s": k * nout * nchans / dt}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(beams or time ranges would be sharded across GPUs with no exchange "
              "beyond a max_delay halo).", file=sys.stderr)
        sys.exit(2)

    if args.summarize_counters:
        summarize_counters(args)
        return

    import torch
    from paper_1201_5380_amd import Plan, synth

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        n = 1 << 30
        a = torch.empty(n, dtype=torch.uint8, device=dev)
        b = torch.empty(n, dtype=torch.uint8, device=dev)
        a.fill_(1)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n, "launches": 5}))
        return

    beam = synth.survey_beam(nsamps=args.nsamps)
    plan = Plan(beam.nchans, beam.dt, beam.f_top, beam.df, beam.nbits).set_dm_list(beam.dms)
    table = plan.delay_table()
    beam.inject(lambda i: table[i])
    packed = beam.packed()
    nsamps, nchans, ndm = beam.nsamps, beam.nchans, len(beam.dms)
    mx = plan.max_delay
    nout = nsamps - mx

    inp = torch.from_numpy(packed.reshape(-1)).to(dev)
    out = torch.empty((ndm, nout), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    tune_ms = None
    if args.tile:
        plan.set_tile_config(tile_arg(args.tile))
    elif not args.no_tune:
        tune_ms = plan.tune(inp, out, nsamps, cache_path=args.tune_cache)
    cfg = plan.tile_config()

    for _ in range(args.warmup):
        plan.execute(inp, nsamps, out=out)
    torch.cuda.synchronize()

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for i in range(args.steps):
        starts[i].record(stream)
        plan.execute(inp, nsamps, out=out, stream=stream)
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    kern_ms = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])

    copies = copy_times(torch, dev, packed, out, ms_per_step=float(np.mean(kern_ms)))

    # sanity: every injected pulse peaks at its trial and time
    got = out.cpu().numpy().view(np.uint32)
    pulses_ok = True
    for p in beam.pulses:
        lo, hi = max(0, p.t0 - 100), min(nout, p.t0 + 101)
        win = got[:, lo:hi]
        dd, tt = np.unravel_index(int(win.argmax()), win.shape)
        pulses_ok &= (int(dd), int(tt) + lo) == (p.dm_index, p.t0)

    outputs = ndm * nout
    adds = outputs * nchans
    mean_ms = float(kern_ms.mean())
    ms_per_step = wall * 1e3 / args.steps
    alg_bytes = nsamps * nchans * beam.nbits // 8 + 4 * outputs + 4 * ndm * nchans
    # counters of the dominant kernel (HBM bytes from rocprofv3 FETCH_SIZE /
    # WRITE_SIZE, VALU issue from SQ_INSTS_VALU and GRBM_GUI_ACTIVE), only while
    # the kernel source and the tile shape are the ones they were taken on
    ctr = counters_for(args.counters_json, beam.name, cfg)
    med_ms = float(np.median(kern_ms))

    result = {
        "metric": "dedispersed outputs/s (DM x sample)",
        "value": outputs / (ms_per_step * 1e-3),
        "unit": "outputs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": f"survey beam: 2-bit, {nchans} ch, {nsamps} samples x 64 us, "
                        f"{ndm} DMs in [0, 1000), f_top 1581.8 MHz, df -0.390625 MHz",
            "nsamps": nsamps, "nchans": nchans, "nbits": beam.nbits, "ndm": ndm,
            "max_delay": mx, "nout": nout, "tile": cfg,
        },
        "kernel_ms": {"runs": args.steps, "mean": mean_ms, "median": med_ms,
                      "p5": float(np.percentile(kern_ms, 5)),
                      "p95": float(np.percentile(kern_ms, 95))},
        "channel_adds_per_s": adds / (med_ms * 1e-3),
        "realtime_factor": nsamps * beam.dt / (med_ms * 1e-3),
        "roofline": roofline_block(beam.nbits, adds, mean_ms, ctr),
        "hbm_algorithmic_GBs": alg_bytes / (mean_ms * 1e-3) / 1e9,
        "hbm_algorithmic_bytes": alg_bytes,
        "pulses_recovered": bool(pulses_ok),
        "tune_best_ms": tune_ms,
        "copies": copies,
        "input_sha256": synth.sha256(packed),
        "gpu": gpu_info(torch),
        "host": host_info(),
    }
    if not args.no_systems:
        del got, out
        leg_steps = min(20, max(3, args.steps // 2))
        legs = {
            "scrunched": lambda: bench_scrunched(torch, dev, plan, inp, nsamps, leg_steps, mean_ms),
            "subband": lambda: bench_subband(torch, dev, plan, inp, nsamps, leg_steps, mean_ms),
            "tree": lambda: bench_tree(torch, dev, beam, inp, nsamps, leg_steps),
            "large_beam": lambda: bench_large(torch, dev, 11, args.counters_json, args.large_tile,
                                              args.tune_cache),
            "tiny": lambda: bench_tiny(torch, dev),
            "batched": lambda: bench_batch(torch, dev, max(3, leg_steps // 2)),
            "serving": lambda: bench_serve(torch, dev, args.serve_seconds),
        }
        for name in [x for x in args.legs.split(",") if x]:
            if name not in legs:
                raise SystemExit(f"unknown leg {name!r}; legs: {', '.join(legs)}")
            torch.cuda.empty_cache()
            result[name] = legs[name]()
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(packed, nsamps, nchans, beam.nbits, table,
                                              args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
