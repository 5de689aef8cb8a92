"""Benchmark of the CPRA hot path on one MI355X.

One step = one whole reconstruction of the 512x512x360 cell-like scan
(N = 512, Np = 360) with inputs already resident in HBM: plan set-up, input
preparation and random initial objects (submit), 200 HIO iterations with
the carousel coupling every 10 iterations, and step D (Fourier-slice
insertion + 3D inverse FFT into a 512^3 volume).  The headline value is
pattern-iterations/s over the whole step: 200 * 360 / step time.

Also reported:
  * roofline of the dominant kernel (HIP events around every column and row
    pass on the plan's stream, algorithmic bytes per launch / mean duration);
  * cpu_baseline: the FP64 oracle on a bounded sample (8 angles x 3
    iterations, single thread) on this machine's host;
  * last-frame-to-volume latency under the serving loop: 8 concurrent scans
    of the same shape whose frames land at 20 frames/s each, reconstructed on
    partial angle sets as they land (about 20 s of wall time; --serve-scans 0
    skips it, --serve-rounds R repeats it for R x 8 samples).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
ROOT = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(ROOT, "paper_2402_05283_amd", "csrc")
TRAFFIC_MD = os.path.join(ROOT, "profiles", "traffic_col_row_n512_np360.md")
COPY_BYTES = 1 << 30           # plain device copy used to calibrate the HBM byte counters

N, NP, ITERS, N_EI, BETA = 512, 360, 200, 10, 0.9


def algorithmic_bytes(N, Np, n_ei, amp_bytes=8, real_bytes=4):
    """Bytes each pass must move per launch, averaged over an episode (the boundary launch's
    extra neighbour reads spread over the n_ei launches of the episode).

    Column pass per angle: read P and write Pmid (N x N/2 complex each) and
    read the amplitude pairs (N x N/2 pairs); at an episode boundary it also
    reads the two neighbours' P.  Row pass per angle: read Pmid, read and
    write the real iterate g, write P, read the support bits; at a boundary
    it also reads the two neighbours' g.
    """
    H = N // 2
    cplane = N * H * 2 * real_bytes
    rplane = N * N * real_bytes
    col = 2 * cplane + N * H * amp_bytes + (2 * cplane) / n_ei
    row = 2 * cplane + 2 * rplane + N * N / 8 + (2 * rplane) / n_ei
    return col * Np, row * Np


def _oracle_child(code, threads, timeout=900):
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1",
               NUMEXPR_NUM_THREADS="1", HIP_VISIBLE_DEVICES="", CUDA_VISIBLE_DEVICES="", ROCR_VISIBLE_DEVICES="")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=timeout)
    if out.returncode != 0:
        return {"error": out.stderr[-500:]}
    return json.loads(out.stdout.strip().splitlines()[-1])


def cpu_baseline(scan):
    """The FP64 oracle on the host, in a child process that never touches the GPU, on two bounded
    samples of the benchmark scan:
      * one thread: angles 0-7 (all present, so the 8 form the coupling ring), 3 HIO iterations
        including one coupling;
      * all cores: a process pool of one worker per core (len(os.sched_getaffinity(0))), each
        running oracle iterations of whole angles (the iterations of an episode are independent
        per angle); 2 angles per worker, 10 HIO iterations each after the coupled start.
    Reported value: the all-core figure."""
    import tempfile
    cores = len(os.sched_getaffinity(0))
    n_all = 2 * cores
    with tempfile.TemporaryDirectory() as td:
        np.save(os.path.join(td, "I.npy"), scan["I"][:max(8, n_all)])
        np.save(os.path.join(td, "S.npy"), scan["support"][:max(8, n_all)])
        single = _oracle_child(f"""
import sys, time, json, numpy as np
sys.path.insert(0, {ROOT!r})
from oracle import cpra as C
I = np.load({os.path.join(td, 'I.npy')!r})[:8]; S = np.load({os.path.join(td, 'S.npy')!r})[:8]
o = C.Oracle({N}, {NP}, seed={scan['phase_seed']}, n_ei={N_EI})
t0 = time.perf_counter()
o.submit(0, I, S)
t1 = time.perf_counter()
o.iterate(3, C.HIO, {BETA})
t2 = time.perf_counter()
print(json.dumps({{"submit_s": t1 - t0, "iter_s": t2 - t1}}))
""", 1)
        pool = _oracle_child(f"""
import sys, time, json, numpy as np
from multiprocessing import get_context
sys.path.insert(0, {ROOT!r})
from oracle import cpra as C
I = np.load({os.path.join(td, 'I.npy')!r}); S = np.load({os.path.join(td, 'S.npy')!r})

def work(n):
    A = C.amplitudes(I[n]); sup = S[n] != 0
    g = C.initial_object(A, {scan['phase_seed']}, n)
    for it in range(10):
        gp = C.inverse_real(C.modulus_projection(C.forward(g), A))
        g = C.real_space_update(g, gp, sup, C.HIO, {BETA}, True, it == 9)
    return float(g.sum())

with get_context("fork").Pool({cores}) as p:
    p.map(work, range({cores}))            # warm the workers
    t0 = time.perf_counter()
    p.map(work, range({n_all}), chunksize=1)
    t1 = time.perf_counter()
print(json.dumps({{"iter_s": t1 - t0}}))
""", cores)
    if "error" in single or "error" in pool:
        return {"error": single.get("error") or pool.get("error")}
    single_v = 8 * 3 / single["iter_s"]
    all_v = n_all * 10 / pool["iter_s"]
    return {"value": round(all_v, 2), "unit": "pattern-iterations/s", "cores": cores, "kind": "oracle",
            "sample": f"N=512 cell scan, {n_all} angles x 10 HIO iterations (each from its random start, "
                      f"the last writing the estimate), one worker process per core, FP64 numpy oracle; "
                      f"{pool['iter_s']:.1f} s wall (also timed: W_0 per angle inside the workers)",
            "single_core": {"value": round(single_v, 2), "cores": 1,
                            "sample": f"angles 0-7 (one coupling ring), 3 HIO iterations incl. one coupling; "
                                      f"{single['iter_s']:.1f} s iterate + {single['submit_s']:.1f} s submit"}}


def kernel_source_hash():
    """SHA-256 over the sources that define the column and row passes and their launches: cx.hpp,
    kernels.hpp and the iteration's launch function in impl.hpp (from `static void step(` to the
    next function)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("cx.hpp", "kernels.hpp"):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(CSRC, "impl.hpp")) as fh:
        src = fh.read()
    a = src.index("  static void step(")
    b = src.index("  static void colerr(", a)
    h.update(src[a:b].encode())
    return h.hexdigest()


def load_traffic():
    """HBM bytes per launch from the committed counter summary, or None when the kernel
    sources have changed since those counters were taken."""
    try:
        with open(TRAFFIC_MD) as fh:
            for line in fh:
                if line.startswith("traffic-json: "):
                    d = json.loads(line[len("traffic-json: "):])
                    return d if d.get("source_sha256") == kernel_source_hash() else None
    except OSError:
        pass
    return None


def roofline_of(col_ms, col_n, row_ms, row_n, n_it, amp_bytes=8, traffic=None):
    """The roofline object of the N=512, Np=360 iteration from the HIP-event totals of the column and
    row passes (col_ms over col_n launches, row_ms over row_n) across n_it timed iterations, and the
    mean iteration time in ms.  A launch covers all 360 angles, or a chunk of them when the tuning
    chose chunk-major order (then each pass takes several launches per iteration): algorithmic bytes
    and counter traffic per launch are scaled by the angles a launch covers.  traffic: the counter
    summary (load_traffic()), or None."""
    col_b360, row_b360 = algorithmic_bytes(N, NP, N_EI, amp_bytes=amp_bytes)
    per_launch = n_it / max(col_n, 1)          # fraction of the 360 angles one launch covers
    col_b, row_b = col_b360 * per_launch, row_b360 * per_launch
    col_avg = col_ms / max(col_n, 1)
    row_avg = row_ms / max(row_n, 1)
    col_gbs = col_b / (col_avg * 1e-3) / 1e9
    row_gbs = row_b / (row_avg * 1e-3) / 1e9
    dom = ("k_col", col_avg, col_gbs, col_b) if col_avg >= row_avg else ("k_row", row_avg, row_gbs, row_b)
    traffic_b = round(traffic[dom[0]]["traffic_bytes"] * per_launch) if traffic else None
    iter_ms = (col_ms + row_ms) / max(n_it, 1)
    it_gbs = (col_b360 + row_b360) / (iter_ms * 1e-3) / 1e9
    full_b = 46.525 * N * N * NP                # full-complex-spectrum byte model (two complex planes per pass)
    other = ("k_row", row_avg, row_gbs) if dom[0] == "k_col" else ("k_col", col_avg, col_gbs)
    roofline = {"bound": "hbm", "achieved": round(dom[2], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(dom[2] / HBM_PEAK_GBS, 4), "traffic": traffic_b, "kernel": dom[0],
                "avg_launch_ms": round(dom[1], 5), "bytes_per_launch": int(dom[3]),
                "launches_per_iteration": round(1.0 / per_launch, 3),
                "other": {"kernel": other[0], "avg_launch_ms": round(other[1], 5), "achieved": round(other[2], 1),
                          "frac": round(other[2] / HBM_PEAK_GBS, 4)},
                "fused_iteration": {"achieved": round(it_gbs, 1), "frac": round(it_gbs / HBM_PEAK_GBS, 4),
                                    "bytes": int(col_b360 + row_b360), "ms": round(iter_ms, 5),
                                    "what": "column + row pass algorithmic bytes over their summed mean "
                                            "launch times: the whole fused FFT + projection iteration"},
                "full_complex_model_frac": round(full_b / (iter_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    return roofline, iter_ms


def _pmc_rows(d):
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    if not rows:
        raise SystemExit(f"no counter_collection.csv under {d}")
    return rows


def summarize_pmc(fetch_dir, write_dir, cmd):
    """Markdown summary of a FETCH_SIZE run and a WRITE_SIZE run of `bench.py --calibrate-copy`:
    per-dispatch HBM bytes of the column and row passes, scaled by what the same counters
    read for the plain 1 GiB device copy."""
    import re

    def per_kernel(rows, counter):
        acc = {}
        for r in rows:
            if r["Counter_Name"] != counter:
                continue
            name = r["Kernel_Name"]
            v = float(r["Counter_Value"]) * 1024.0      # counters are KiB per dispatch
            if "copyBuffer" in name and v > COPY_BYTES / 2:
                key = "copy"
            else:
                if re.search(r"cpra::k_row<512, float\b", name):
                    key = "k_row"
                elif re.search(r"cpra::k_col(_pair)?<512, float, [^,]+, 2u>, 0,", name):
                    key = "k_col"                          # iteration column pass (not the initial guess)
                else:
                    continue
            acc.setdefault(key, []).append(v)
        return acc

    fetch = per_kernel(_pmc_rows(fetch_dir), "FETCH_SIZE")
    write = per_kernel(_pmc_rows(write_dir), "WRITE_SIZE")
    if "copy" not in fetch or "copy" not in write:
        raise SystemExit("the 1 GiB calibration copy is missing from the counter runs")
    ff = COPY_BYTES / (sum(fetch["copy"]) / len(fetch["copy"]))
    fw = COPY_BYTES / (sum(write["copy"]) / len(write["copy"]))
    col_b, row_b = algorithmic_bytes(N, NP, N_EI)
    model = {"k_col": col_b, "k_row": row_b}
    out = {"source_sha256": kernel_source_hash(), "fetch_factor": ff, "write_factor": fw}
    lines = ["# HBM traffic of the column and row passes: N=512, Np=360 cell scan", "",
             "Commands (repo root, one MI355X; one counter per run):", "",
             f"    {cmd.format(counter='FETCH_SIZE', out=fetch_dir)}",
             f"    {cmd.format(counter='WRITE_SIZE', out=write_dir)}",
             f"    python3 bench.py --summarize-pmc {fetch_dir} {write_dir}", "",
             f"Calibration: a plain device copy of {COPY_BYTES >> 20} MiB reads "
             f"{sum(fetch['copy']) / len(fetch['copy']) / 2**20:.1f} MiB on FETCH_SIZE and "
             f"{sum(write['copy']) / len(write['copy']) / 2**20:.1f} MiB on WRITE_SIZE, so fetches are scaled "
             f"by {ff:.3f} and writes by {fw:.3f}.", "",
             "| Kernel (per 360-angle launch, all iteration launches) | Launches | Fetch (GB) | Write (GB) | "
             "HBM total (GB) | Algorithmic (GB) | Ratio |", "|---|---|---|---|---|---|---|"]
    for k in ("k_col", "k_row"):
        fb = ff * sum(fetch[k]) / len(fetch[k])
        wb = fw * sum(write[k]) / len(write[k])
        out[k] = {"fetch_bytes": fb, "write_bytes": wb, "traffic_bytes": fb + wb, "launches": len(fetch[k])}
        lines.append(f"| {k} | {len(fetch[k])} | {fb / 1e9:.3f} | {wb / 1e9:.3f} | {(fb + wb) / 1e9:.3f} | "
                     f"{model[k] / 1e9:.3f} | {(fb + wb) / model[k]:.3f} |")
    lines += ["", "The line below is read by bench.py, which reports `traffic` only while the kernel "
              "sources hash to the same value.", "", "traffic-json: " + json.dumps(out)]
    return "\n".join(lines) + "\n"


def summarize_sq(sq_dir, cmd):
    """Markdown summary of a rocprofv3 --pmc run of SQ counters: per kernel of the iteration and of
    step D, VALU instructions per wave, the share of wave time spent waiting on instruction
    dependencies (SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES) and issuing VALU (SQ_ACTIVE_INST_VALU /
    SQ_WAVE_CYCLES), and the average resident waves per CU (SQ_WAVE_CYCLES counts every 4 cycles,
    GRBM_GUI_ACTIVE sums the 8 XCDs)."""
    import re
    acc = {}
    for r in _pmc_rows(sq_dir):
        m = re.search(r"cpra::(k_col_pair|k_row|k_stepd_stage|k_stepd_gather|k_stepd_heavy|k_stepd_rows|k_stepd_cols)"
                      r"<512, float[^(]*?(?:, (true|false))?[,>]",
                      r["Kernel_Name"])
        if not m:
            continue
        name = r["Kernel_Name"]
        key = m.group(1)
        if key == "k_col_pair":
            if ", 0, false, false>" not in name:
                continue
        if key == "k_row":
            if "false" not in name.split("k_row<")[1].split(">")[0]:
                continue
        acc.setdefault(key, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    lines = ["# SQ counters of the iteration and step-D kernels: N=512, Np=360 cell scan", "",
             "Command (repo root, one MI355X):", "", f"    {cmd}", "",
             "Per launch averages (plain column and row passes: no coupling, no error history).  "
             "VALU busy = VALU instructions x 4 cycles / (1024 SIMDs x launch cycles).", "",
             "| Kernel | Launches | Waves | VALU instr / wave | Dependency waits / wave time | VALU issue / wave time | "
             "Waves resident per CU | VALU busy |", "|---|---|---|---|---|---|---|---|"]
    for k in ("k_col_pair", "k_row", "k_stepd_stage", "k_stepd_gather", "k_stepd_heavy", "k_stepd_rows", "k_stepd_cols"):
        a = acc.get(k)
        if not a:
            continue
        mean = {c: sum(v) / len(v) for c, v in a.items()}
        w = mean["SQ_WAVES"]
        cyc = mean["GRBM_GUI_ACTIVE"] / 8.0
        resident = 4.0 * mean["SQ_WAVE_CYCLES"] / (256.0 * cyc)
        busy = mean["SQ_INSTS_VALU"] * 4.0 / (1024.0 * cyc)
        lines.append(f"| {k} | {len(a['SQ_WAVES'])} | {w:.0f} | {mean['SQ_INSTS_VALU'] / w:.0f} | "
                     f"{mean['SQ_WAIT_INST_ANY'] / mean['SQ_WAVE_CYCLES']:.2f} | "
                     f"{mean['SQ_ACTIVE_INST_VALU'] / mean['SQ_WAVE_CYCLES']:.2f} | {resident:.1f} | {busy:.2f} |")
    return "\n".join(lines) + "\n"


def summarize_trace(trace_dir, bench_json, cmd):
    """Markdown summary of a `rocprofv3 --kernel-trace --stats` run of bench.py, beside the
    launch durations that bench.py measured itself with HIP events in the same run."""
    import csv
    import glob
    files = glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no kernel_stats.csv under {trace_dir}")
    with open(files[0]) as fh:
        rows = list(csv.DictReader(fh))
    with open(bench_json) as fh:
        b = json.loads([l for l in fh if l.startswith("{")][-1])
    r = b["roofline"]
    ev = {r["kernel"]: r["avg_launch_ms"], r["other"]["kernel"]: r["other"]["avg_launch_ms"]}
    lines = ["# Kernel-trace summary: N=512, Np=360 cell scan, whole reconstruction per step", "",
             "Command (repo root, one MI355X):", "", f"    {cmd}", "",
             f"Each step: plan set-up, submit of 360 angles (prep + initial objects), {b['config']['iterations']} "
             f"HIO iterations (coupling every {b['config']['n_ei']}), step D into a 512^3 volume.  "
             f"Besides the headline, only the FP16-amplitude leg (the `__half2` column passes) and the "
             f"error-history leg run (no comparison, schedule, batch or serving legs); the row pass is the "
             f"same kernel for both amplitude types.  "
             f"bench.py in the same run: value {b['value']:.0f} pattern-iterations/s, {b['ms_per_step']:.1f} ms "
             f"per step; HIP-event mean launch time k_col {ev.get('k_col', 0) * 1e3:.1f} us, "
             f"k_row {ev.get('k_row', 0) * 1e3:.1f} us.", "",
             "| Kernel | Calls | Total ms | Avg us | % |", "|---|---|---|---|---|"]
    for x in rows:
        lines.append(f"| `{x['Name'][:110]}` | {x['Calls']} | {float(x['TotalDurationNs']) / 1e6:.2f} | "
                     f"{float(x['AverageNs']) / 1e3:.1f} | {float(x['Percentage']):.1f} |")
    return "\n".join(lines) + "\n"


def serving_sources(torch, scan512, cache):
    """Frame sources of the serving mix, as device tensors (I, S) per (N, Np): the benchmark's
    512^3 cell scan with Poisson noise at 1e6 photons peak, the 256^3 polyhedron scan (Poisson 1e6)
    and a 1024 scan of five ellipsoids (Poisson 1e6).  A 180-angle scan of N = 256 or 512 takes the
    even angles of the 360-angle scan (the same angles pi n / 180).  The 1024 source has 180
    angles only: its projections at 1024^2 take minutes of host time per 360 angles."""
    from synth import make_scan
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(4000 + 1)
    I = scan512["I"].astype(np.float64)
    peak = 1e6 / I.reshape(I.shape[0], -1).max(axis=1)
    I512 = rng.poisson(I * peak[:, None, None]).astype(np.float32)
    if 256 not in cache:
        print("[bench] serving: generating the N=256 source scan", file=sys.stderr, flush=True)
        cache[256] = make_scan(2, N=256, Np=360)
    print("[bench] serving: generating the N=1024 source scan", file=sys.stderr, flush=True)
    s1024 = make_scan(1, N=1024, Np=180, peak=1e6)
    src = {}
    for n, (Iv, Sv) in ((512, (I512, scan512["support"])), (256, (cache[256]["I"], cache[256]["support"]))):
        It, St = torch.from_numpy(Iv).to(dev), torch.from_numpy(Sv).to(dev)
        src[(n, 360)] = (It, St)
        src[(n, 180)] = (It[0::2].contiguous(), St[0::2].contiguous())
    src[(1024, 180)] = (torch.from_numpy(s1024["I"]).to(dev), torch.from_numpy(s1024["support"]).to(dev))
    return src


def serving_latency(cp, torch, scan, I, S, args, cache):
    """Last-frame-to-volume latency under the serving loop on a mix of scan shapes: `serve_scans`
    detector lanes, each delivering scans back to back (0.25 s apart, lanes staggered by 0.25 s);
    every scan's shape is drawn (seeded) from N in {256, 512, 1024} and N_p in {180, 360} (N = 1024
    with 180 only), its frames land at serve_fps in angle order; each landed frame earns 10 HIO
    iterations on the partial angle set (one episode), the last one 50 more, then step D.  The
    scans of all lanes that are open at a time are served together (continuous batching)."""
    from paper_2402_05283_amd import serve
    src = serving_sources(torch, scan, cache)
    rng = np.random.default_rng(5)
    jobs = []
    for lane in range(args.serve_scans):
        t = 0.25 * lane
        for i in range(args.serve_per_lane):
            n = int(rng.choice([256, 512, 1024]))
            npp = 180 if n == 1024 else int(rng.choice([180, 360]))
            It, St = src[(n, npp)]
            jobs.append(serve.Job(t, n, npp, (lambda k, It=It, St=St: (It[k:k + 1], St[k:k + 1])), args.serve_fps,
                                  seed=scan["phase_seed"] + 1 + len(jobs), theta=np.pi * np.arange(npp) / npp))
            t += npp / args.serve_fps + 0.25
    T = max(j.t_start + j.Np / j.fps for j in jobs)
    srv = serve.Server(200 << 30, n_ei=N_EI, r_frame=N_EI, r_final=50, algo=cp.HIO, beta=BETA,
                       hold_others=not args.serve_no_hold, depth=args.serve_depth)
    prev_fuse = cp.set_batch_fusion(args.serve_fusion) if args.serve_fusion is not None else None
    print(f"[bench] serving {len(jobs)} scans on {args.serve_scans} lanes at {args.serve_fps} frames/s each "
          f"(~{T:.0f} s)", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    count = [0]

    def on_done(sc):
        count[0] += 1
        print(f"[bench] serving: {count[0]}/{len(jobs)} scans done (N={sc.N} Np={sc.Np}), last-frame-to-volume "
              f"{sc.latency_s * 1e3:.1f} ms", file=sys.stderr, flush=True)
    done = serve.replay(srv, jobs, on_done=on_done)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fuse = cp.get_batch_fusion()
    if prev_fuse is not None:
        cp.set_batch_fusion(prev_fuse)
    lat = np.array([d.latency_s for d in done]) * 1e3
    work = sum(d.iters_done * d.Np for d in done)
    print(f"[bench] serving done in {wall:.1f} s; latency p50 {np.percentile(lat, 50):.1f} ms, "
          f"max {lat.max():.1f} ms", file=sys.stderr, flush=True)
    worst = []
    for i in np.argsort(-lat)[:5]:
        d = done[i]
        ms = lambda t: None if t is None else round((t - d.t_last_frame) * 1e3, 1)
        worst.append({"N": d.N, "Np": d.Np, "latency_ms": round(float(lat[i]), 1), "last_submit_ms": ms(d.t_last_submit),
                      "last_issue_ms": ms(d.t_last_issue), "step_d_issue_ms": ms(d.t_assemble)})
    by_shape = {}
    for d, l in zip(done, lat):
        by_shape.setdefault(f"N={d.N},Np={d.Np}", []).append(l)
    del src
    torch.cuda.empty_cache()
    return {"p50": round(float(np.percentile(lat, 50)), 2), "p99": round(float(np.percentile(lat, 99)), 2),
            "max": round(float(lat.max()), 2), "samples": int(lat.size),
            "by_shape": {k: {"samples": len(v), "p50": round(float(np.percentile(v, 50)), 2),
                             "p99": round(float(np.percentile(v, 99)), 2)} for k, v in sorted(by_shape.items())},
            "what": f"last frame to volume ready: {args.serve_scans} lanes of scans back to back, shapes drawn from "
                    f"N in {{256, 512, 1024}}, N_p in {{180, 360}} (1024 with 180), Poisson 1e6 data, "
                    f"{args.serve_fps:g} frames/s per scan, 10 HIO iterations per landed frame (partial angle sets), "
                    f"50 after the last, then step D",
            "shared_launches_up_to_N": fuse, "hold_others": srv.hold_others, "depth": srv.depth,
            "worst": worst, "longest_round_ms": round(srv.step_max_s * 1e3, 1), "rounds_over_50ms": int(srv.slow_steps),
            "serving_wall_s": round(wall, 2), "pattern_iterations": int(work),
            "pattern_iterations_per_s": round(work / wall, 1)}


class Quality:
    """Quality of a scan's objects against the known object: median over angles of E_F; twin
    consistency (the fraction of angles whose estimate is nearer the true projection than its point
    reflection, which fits the same intensities, or one minus it if larger); and the relative L2
    error of the step-D volume against the step-D volume of the true projections, after choosing
    the better of the volume and its twin."""

    def __init__(self, cp, torch, scan, I, S):
        self.torch = torch
        self.Np, self.N = scan["Np"], scan["N"]
        self.A_nat = torch.fft.ifftshift(torch.sqrt(torch.clamp(I, min=0.0)), dim=(-2, -1))
        self.den = (self.A_nat.double() ** 2).sum((-2, -1))
        self.po = torch.from_numpy(scan["po"].astype(np.float32)).to(I.device)
        self.vp = cp.Plan(self.N, self.Np, theta=scan["theta"], n_ei=N_EI, seed=scan["phase_seed"])
        self.vp.submit(0, I, S)
        self.vp.iterate(N_EI, cp.HIO, BETA)                 # step D needs an episode end
        self.v_true = self.vol_of(self.po).clone()

    @staticmethod
    def twin(x, dims):
        for d in dims:
            x = torch_roll_flip(x, d)
        return x

    def vol_of(self, obj):
        self.vp.load_objects(obj)
        return self.vp.assemble_volume()

    def volume_error(self, v):
        t = self.torch
        ve = min(float(t.linalg.norm(v - self.v_true)), float(t.linalg.norm(self.twin(v, (0, 1, 2)) - self.v_true)))
        return round(ve / float(t.linalg.norm(self.v_true)), 4)

    def __call__(self, obj, vol=None):
        t = self.torch
        Np = self.Np
        err = t.empty(Np, dtype=t.float64, device=obj.device)
        near_true = 0
        for c0 in range(0, Np, 60):
            o = obj[c0:c0 + 60]
            G = t.fft.fft2(o)
            err[c0:c0 + 60] = t.sqrt(((G.abs() - self.A_nat[c0:c0 + 60]) ** 2).double().sum((-2, -1))
                                     / self.den[c0:c0 + 60])
            p = self.po[c0:c0 + 60]
            d0 = ((o - p) ** 2).sum((-2, -1))
            d1 = ((o - self.twin(p, (-2, -1))) ** 2).sum((-2, -1))
            near_true += int((d0 < d1).sum())
        v = self.vol_of(obj) if vol is None else vol
        frac = near_true / Np
        return {"median_error": round(float(err.median()), 5), "twin_consistency": round(max(frac, 1 - frac), 4),
                "volume_error": self.volume_error(v)}


def torch_roll_flip(x, d):
    """Point reflection about the centred origin along axis d (index i -> (N - i) mod N)."""
    import torch
    return torch.roll(torch.flip(x, (d,)), 1, d)


def plain_comparison(cp, torch, scan, I, S, args, cpra_iter_ms, Q):
    """CPRA against the plain per-angle method on the same GPU.

    Plain method = the same 2D HIO with no carousel coupling (alpha = (0, 1, 0)): each angle is
    reconstructed on its own.  Two measures of the result after 200 iterations:
      * data fit: median over angles of E_F of the final episode estimates;
      * 3D consistency: the fraction of angles whose estimate is nearer the true projection than
        its twin (the point reflection, which fits the same intensities), and the relative L2
        error of the step-D volume against the step-D volume of the true projections (after
        choosing the better of the volume and its twin).
    Three forms of the plain method are timed: (a) the project's kernels, all angles batched in
    one plan, also run on until its median E_F reaches CPRA's (at most 1000 iterations); (b) a
    straightforward unfused PyTorch version (torch.fft, i.e. rocFFT, over all angles at once,
    elementwise projection and HIO update), from the same initial objects; (c) the project's
    kernels at batch 1, one plan per angle, over a sample of angles."""
    Np, N = scan["Np"], scan["N"]
    th = scan["theta"]
    A_nat, den = Q.A_nat, Q.den
    Sb = S.bool()

    def quality(obj, _vol_of=None):
        return Q(obj)

    def plan(alpha, wrap, n=None):
        th_ = th if n is None else th[n:n + 1]
        p = cp.Plan(N, len(th_), theta=th_, alpha=alpha, wrap=wrap, n_ei=N_EI, seed=scan["phase_seed"])
        if n is None:
            p.submit(0, I, S)
        else:
            p.submit(0, I[n:n + 1], S[n:n + 1])
        return p

    vol_of = Q.vol_of
    out = {}
    pc = plan((0.2, 0.6, 0.2), cp.WRAP_MIRROR)
    pc.iterate(ITERS, cp.HIO, BETA)
    q_cpra = quality(pc.objects(), vol_of)
    del pc
    out["cpra"] = dict(iterations=ITERS, seconds=round(ITERS * cpra_iter_ms * 1e-3, 4), **q_cpra)

    # (a) plain, project kernels, batched over angles
    pp = plan((0.0, 1.0, 0.0), cp.WRAP_PLAIN)
    w0 = pp.objects().clone()
    k, hist, reached, elapsed, q200 = 0, [], None, 0.0, None
    while k < 1000:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pp.iterate(50, cp.HIO, BETA)
        torch.cuda.synchronize()
        elapsed += time.perf_counter() - t0
        k += 50
        q = quality(pp.objects(), vol_of) if k == ITERS else None
        if q is not None:
            q200 = q
        e = q["median_error"] if q else quality_error_only(torch, pp.objects(), A_nat, den)
        hist.append((k, round(e, 5)))
        if reached is None and e <= q_cpra["median_error"]:
            reached = k
        if reached is not None and k >= ITERS:
            break
    del pp
    out["plain_batched"] = dict(at_200=q200, error_history=hist, iterations_to_cpra_error=reached,
                                seconds_per_iteration=round(elapsed / k, 6),
                                seconds_to_cpra_error=None if reached is None else round(elapsed / k * reached, 4))

    # (b) plain, unfused torch.fft, from the same initial objects
    g = w0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(ITERS):
        G = torch.fft.fft2(g)
        mag = G.abs()
        # (|G| = 0 exactly does not occur on these scans; its zero-phase value is not special-cased)
        Gp = G * (A_nat / torch.clamp(mag, min=1e-30))
        gp = torch.fft.ifft2(Gp).real
        gam = Sb & (gp >= 0)
        if (it + 1) % N_EI == 0:
            g = torch.where(gam, gp, torch.zeros_like(gp))
        else:
            g = torch.where(gam, gp, g - BETA * gp)
    torch.cuda.synchronize()
    t_torch = time.perf_counter() - t0
    del G, Gp, gp, mag, gam
    out["plain_torch_fft"] = dict(pattern_iterations_per_s=round(ITERS * Np / t_torch, 1), at_200=quality(g, vol_of),
                                  what="torch.fft.fft2/ifft2 (rocFFT) over all angles at once, elementwise "
                                       "projection and HIO in torch, complex64")
    del g

    # (c) plain, project kernels, batch 1 (one plan per angle) over a sample of angles
    sample = list(range(0, Np, 10))
    plans = [plan((0.0, 1.0, 0.0), cp.WRAP_PLAIN, n) for n in sample]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p in plans:
        p.iterate(ITERS, cp.HIO, BETA)
    torch.cuda.synchronize()
    t_b1 = time.perf_counter() - t0
    del plans
    out["plain_batch1_loop"] = {"pattern_iterations_per_s": round(ITERS * len(sample) / t_b1, 1),
                                "angles_timed": len(sample)}
    return out


def paper_schedule(cp, torch, scan, I, S, args, Q):
    """The paper's own schedule on the same scan: N_r = 100 random guesses held at once, step A
    (N_i^pre = 500 HIO iterations of PO 1), step B as the consecutive sweep (N_e = 1, N_ei = 2, the
    paper's timing configuration), step C (merge of the N_l = 10 best guesses) and step D.
    Sequential over angles, parallel over guesses."""
    R, n_pre, n_e, n_ei, n_best = args.guesses, 500, 1, 2, 10
    t = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = cp.Plan(N, NP, n_ei=n_ei, seed=scan["phase_seed"], n_guess=R)
    plan.submit(0, I, S)
    torch.cuda.synchronize()
    t["submit"] = time.perf_counter() - t0
    for name, fn in (("step_A", lambda: plan.prereconstruct(n_pre, cp.HIO, BETA)),
                     ("step_B", lambda: plan.sweep(n_e, cp.HIO, BETA)),
                     ("step_C", lambda: plan.merge(n_best)),
                     ("step_D", lambda: plan.assemble_volume())):
        t1 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        t[name] = time.perf_counter() - t1
        if name == "step_C":
            kept, inv = out
        if name == "step_D":
            vol = out
    total = sum(t.values())
    print("[bench] paper schedule: quality of the merged reconstruction", file=sys.stderr, flush=True)
    merged = plan.objects()[0] if R > 1 else plan.objects()
    qual = Q(merged, vol)
    del merged, vol
    pits = R * (n_pre + NP * n_e * n_ei)
    del plan
    torch.cuda.empty_cache()
    return {"guesses": R, "n_pre": n_pre, "episodes": n_e, "n_ei": n_ei, "n_best": n_best,
            "seconds": {k: round(v, 4) for k, v in t.items()}, "total_s": round(total, 3),
            "pattern_iterations": pits,
            "pattern_iterations_per_s_steps_AB": round(pits / (t["step_A"] + t["step_B"]), 1),
            "kept": [int(k) for k in kept], "inverted": [bool(i) for i in inv],
            "merged_quality": qual}


def variants(cp, torch, scan, I, S, args):
    """The algorithm variants on the same scan and kernels, timed on their own: 200 RAAR
    iterations (beta 0.9); 200 HIO iterations with five coupling taps (a coupling pass of its own
    at each of the 20 boundaries); one shrinkwrap support update (sigma 2, threshold 0.1); step D
    with bilinear and with nearest insertion (first call with the host-built tables, then step D
    alone); the 3D refinement after step D (50 error-reduction iterations, 3D shrinkwrap every 5;
    step D and its tables included)."""
    out = {}

    def run(name, plan_kw, body):
        plan = cp.Plan(N, NP, n_ei=N_EI, seed=scan["phase_seed"], **plan_kw)
        plan.submit(0, I, S)
        plan.iterate(N_EI, cp.HIO, BETA)                 # reach an episode end first
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = body(plan)
        torch.cuda.synchronize()
        out[name] = dict(seconds=round(time.perf_counter() - t0, 5), **(res or {}))
        del plan

    run("raar_200", {}, lambda p: (p.iterate(ITERS, cp.RAAR, BETA), None)[1])
    out["raar_200"]["pattern_iterations_per_s"] = round(ITERS * NP / out["raar_200"]["seconds"], 1)
    run("hio_200_five_taps", {"taps": (0.05, 0.15, 0.6, 0.15, 0.05)}, lambda p: (p.iterate(ITERS, cp.HIO, BETA), None)[1])
    out["hio_200_five_taps"]["pattern_iterations_per_s"] = round(ITERS * NP / out["hio_200_five_taps"]["seconds"], 1)
    run("shrinkwrap", {}, lambda p: (p.shrinkwrap(2.0, 0.1), None)[1])
    vol = torch.empty((N, N, N), dtype=torch.float32, device=I.device)

    def step_d(p):
        # the first call builds the insertion tables on the host (the stream is idle here, so
        # nothing hides it); the second is step D alone
        t = time.perf_counter()
        p.assemble_volume(vol)
        torch.cuda.synchronize()
        first = time.perf_counter() - t
        t = time.perf_counter()
        p.assemble_volume(vol)
        torch.cuda.synchronize()
        return {"step_d_s": round(time.perf_counter() - t, 5), "first_call_s": round(first, 5)}

    run("step_d_bilinear", {"insertion": cp.INSERT_BILINEAR}, step_d)
    run("step_d_nearest", {}, step_d)
    run("refine_50_shrink5", {}, lambda p: (p.refine_volume(50, shrink_every=5, sigma=2.0, threshold=0.1, out=vol),
                                            None)[1])
    del vol
    return out


def batched_scans(cp, torch, scan512, args, cache):
    """Config-3-like batch: 48 scans of uneven size (N drawn from {128, 192, 256, 384, 512}, N_p
    from [90, 360], seeded), 300 HIO iterations each, advanced together through
    cpra_iterate_batch (every plan on its own stream), against the same plans iterated one after
    another.  Frames come from one synthetic scan per N (the bench scan for N = 512), each plan
    taking a seeded subset of its angles and its own phase seed."""
    from synth import make_scan
    rng = np.random.default_rng(3)
    sizes = rng.choice([128, 192, 256, 384, 512], size=args.batch_scans)
    nps = rng.integers(90, 361, size=args.batch_scans)
    src = {512: scan512}
    for n in sorted(set(int(x) for x in sizes) - {512}):
        print(f"[bench] batched: generating the N={n} source scan", file=sys.stderr, flush=True)
        if n not in cache:
            cache[n] = make_scan(2 if n >= 256 else 1, N=n, Np=360)
        src[n] = cache[n]
    dev = torch.device("cuda", 0)
    data = {n: (torch.from_numpy(s["I"]).to(dev), torch.from_numpy(s["support"]).to(dev), s["theta"])
            for n, s in src.items()}

    def make_plans(streams):
        plans = []
        for i, (n, npp) in enumerate(zip(sizes, nps)):
            n, npp = int(n), int(npp)
            I, S, th = data[n]
            idx = np.sort(rng_sub.choice(360, size=npp, replace=False))
            it = torch.from_numpy(idx).to(dev)
            p = cp.Plan(n, npp, theta=th[idx], n_ei=N_EI, seed=1000 + i, stream=streams[i] if streams else None)
            p.submit(0, I.index_select(0, it).contiguous(), S.index_select(0, it).contiguous())
            plans.append(p)
        torch.cuda.synchronize()
        return plans

    iters = args.batch_iters
    work = int(iters * nps.sum())
    rng_sub = np.random.default_rng(4)
    plans = make_plans(None)
    t0 = time.perf_counter()
    for p in plans:
        p.iterate(iters, cp.HIO, BETA)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    del plans
    t_bat = {}
    for fuse in (0, 256, 1024):
        rng_sub = np.random.default_rng(4)
        streams = [torch.cuda.Stream() for _ in sizes]
        plans = make_plans(streams)
        prev = cp.set_batch_fusion(fuse)
        t0 = time.perf_counter()
        cp.iterate_batch(plans, iters, cp.HIO, BETA)
        torch.cuda.synchronize()
        t_bat[fuse] = time.perf_counter() - t0
        cp.set_batch_fusion(prev)
        del plans
        torch.cuda.empty_cache()
    best = min(t_bat, key=t_bat.get)
    return {"scans": int(args.batch_scans), "iterations": iters, "pattern_iterations": work,
            "sizes": {int(n): int((sizes == n).sum()) for n in sorted(set(int(x) for x in sizes))},
            "batched_s": round(t_bat[best], 3), "sequential_s": round(t_seq, 3),
            "batched_pattern_iterations_per_s": round(work / t_bat[best], 1),
            "sequential_pattern_iterations_per_s": round(work / t_seq, 1),
            "by_fusion": {f"fuse_N<={k}": {"s": round(v, 3), "pattern_iterations_per_s": round(work / v, 1)}
                          for k, v in t_bat.items()},
            "what": "cpra_iterate_batch over all 48 plans, each on its own stream; plans of one size class with "
                    "N <= the fusion limit share one launch per pass per iteration (limit 0: every plan's "
                    "launches interleaved on its own stream); batched_s is the best limit; sequential: "
                    "cpra_iterate on each plan in turn"}


def fp16_leg(cp, torch, scan, I, S, vol, stream, args, steps=3):
    """The headline step with FP16 amplitude storage (per-angle power-of-two scale): whole-step
    throughput and the mean iteration time from HIP events."""
    def one(timed):
        plan = cp.Plan(N, NP, n_ei=N_EI, amp=cp.AMP_F16, seed=scan["phase_seed"], stream=stream)
        if timed:
            plan.set_kernel_timing(True)
        plan.submit(0, I, S)
        plan.iterate(ITERS, cp.HIO, BETA)
        plan.assemble_volume(vol)
        res = plan.kernel_timing() if timed else None
        torch.cuda.synchronize()
        return res
    one(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c = r = 0.0
    n = 0
    for _ in range(steps):
        cm, cn, rm, rn = one(True)
        c += cm; r += rm; n += cn
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    it = (c + r) / max(n, 1)
    col_b, row_b = algorithmic_bytes(N, NP, N_EI, amp_bytes=4)
    return {"value": round(ITERS * NP / dt, 1), "unit": "pattern-iterations/s", "ms_per_step": round(dt * 1e3, 3),
            "steps": steps, "ms_per_iteration": round(it, 4),
            "fused_iteration_frac": round((col_b + row_b) / (it * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "what": "same step as the headline with amplitudes stored as binary16 pairs times a per-angle "
                    "power-of-two scale (error against the FP64 oracle: tests/test_gpu_parity.py "
                    "precision study, tests/test_gpu_noisy.py)"}


def error_history_leg(cp, torch, scan, I, S, stream, iter_ms):
    """Cost of recording E_F for every angle and iteration: 200 iterations with the error history
    (FP64 partials per tile, fixed-order reduction, copied to the host every 64 iterations)."""
    plan = cp.Plan(N, NP, n_ei=N_EI, seed=scan["phase_seed"], stream=stream)
    plan.submit(0, I, S)
    plan.iterate(N_EI, cp.HIO, BETA, errors=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e = plan.iterate(ITERS, cp.HIO, BETA, errors=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / ITERS
    return {"ms_per_iteration": round(dt * 1e3, 4), "without_ms_per_iteration": round(iter_ms, 4),
            "final_median_error": round(float(np.median(e[-1])), 5),
            "what": "wall time per iteration of cpra_iterate with err_out over 200 iterations (host "
                    "synchronisation every 64 iterations included), against the HIP-event iteration time "
                    "without it"}


def quality_error_only(torch, obj, A_nat, den):
    err = []
    for c0 in range(0, obj.shape[0], 60):
        G = torch.fft.fft2(obj[c0:c0 + 60])
        err.append(torch.sqrt(((G.abs() - A_nat[c0:c0 + 60]) ** 2).double().sum((-2, -1)) / den[c0:c0 + 60]))
    return float(torch.cat(err).median())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--amp16", action="store_true", help="FP16 amplitude storage")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="run the headline plans with the library's default launch choices")
    ap.add_argument("--iters", type=int, default=ITERS)
    ap.add_argument("--serve-scans", type=int, default=8, help="detector lanes of the serving leg (0: skip)")
    ap.add_argument("--serve-per-lane", type=int, default=13,
                    help="scans per lane (latency samples = lanes x scans per lane)")
    ap.add_argument("--serve-depth", type=int, default=1,
                    help="serving: episodes in flight per scan before its last frame has landed")
    ap.add_argument("--serve-no-hold", action="store_true",
                    help="serving: other scans keep issuing while a scan whose last frame has landed is unfinished")
    ap.add_argument("--serve-fps", type=float, default=20.0, help="frames per second per scan")
    ap.add_argument("--serve-fusion", type=int, default=None,
                    help="size limit of shared launches in the serving leg (cpra_set_batch_fusion; default: "
                         "the library's)")
    ap.add_argument("--no-compare", action="store_true", help="skip the plain per-angle comparison")
    ap.add_argument("--guesses", type=int, default=100, help="N_r of the paper-schedule leg (0: skip it)")
    ap.add_argument("--batch-scans", type=int, default=48, help="scans of the uneven-size batch leg (0: skip)")
    ap.add_argument("--batch-iters", type=int, default=300)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (the byte-counter calibration)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="print the traffic summary of two rocprofv3 --pmc runs and exit")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("TRACE_DIR", "BENCH_JSON"),
                    help="print the kernel-trace summary of a rocprofv3 --stats run and exit")
    ap.add_argument("--summarize-sq", metavar="SQ_DIR", help="print the SQ-counter summary of a rocprofv3 --pmc run")
    args = ap.parse_args()
    if args.summarize_trace:
        tdir, tjson = args.summarize_trace
        cmd = (f"rocprofv3 --kernel-trace --stats --output-format csv -d {tdir} -o run "
               "-- python3 bench.py --steps 2 --warmup 1 --no-cpu-baseline --no-compare --guesses 0 --serve-scans 0 --batch-scans 0 "
               f"--no-autotune > {tjson}")
        print(summarize_trace(*args.summarize_trace, cmd), end="")
        return
    if args.summarize_sq:
        cmd = ("timeout -s KILL 180 rocprofv3 --pmc SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_ACTIVE_INST_VALU "
               "SQ_WAIT_INST_ANY SQ_INSTS_VMEM_RD SQ_INSTS_VALU SQ_WAIT_ANY GRBM_GUI_ACTIVE --output-format csv "
               f"-d {args.summarize_sq} -o run -- python3 bench.py --steps 1 --warmup 0 --iters 20 --no-cpu-baseline "
               "--serve-scans 0 --no-compare --guesses 0 --batch-scans 0 --no-autotune")
        print(summarize_sq(args.summarize_sq, cmd), end="")
        return
    if args.summarize_pmc:
        cmd = ("timeout -s KILL 120 rocprofv3 --pmc {counter} --output-format csv -d {out} -o run "
               "-- python3 bench.py --steps 1 --warmup 0 --iters 20 --no-cpu-baseline --serve-scans 0 --no-compare "
               "--guesses 0 --batch-scans 0 --no-autotune --calibrate-copy")
        print(summarize_pmc(*args.summarize_pmc, cmd), end="")
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on exactly one GPU (sharding across GPUs is described, not "
              "implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2402_05283_amd as cp
    from synth import make_scan

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    print(f"[bench] generating the N={N} Np={NP} scan", file=sys.stderr, flush=True)
    t = time.time()
    scan = make_scan(4, keep_po=True)
    print(f"[bench] scan ready in {time.time() - t:.1f} s", file=sys.stderr, flush=True)
    I = torch.from_numpy(scan["I"]).to(dev)
    S = torch.from_numpy(scan["support"]).to(dev)
    vol = torch.empty((N, N, N), dtype=torch.float32, device=dev)
    amp = cp.AMP_F16 if args.amp16 else cp.AMP_F32
    stream = torch.cuda.current_stream(dev)

    if args.calibrate_copy:
        src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    tuning = None
    if not args.no_autotune:
        print("[bench] autotuning the launch choices of the N=512 Np=360 shape", file=sys.stderr, flush=True)
        tuning = cp.autotune(N, NP, n_iter=20, n_ei=N_EI, stream=stream)
        print(f"[bench] tuning: {tuning}", file=sys.stderr, flush=True)

    col_ms = row_ms = 0.0
    col_n = row_n = 0
    lat = []
    qcache = []
    src_cache = {}      # synthetic source scans shared by the batch and serving legs

    def quality_of():
        if not qcache:
            qcache.append(Quality(cp, torch, scan, I, S))
        return qcache[0]

    def one_step(timed):
        nonlocal col_ms, row_ms, col_n, row_n
        t0 = time.perf_counter()
        plan = cp.Plan(N, NP, n_ei=N_EI, amp=amp, seed=scan["phase_seed"], stream=stream)
        if timed:
            if tuning and tuning["graphs"]:
                # per-pass event timing needs launch-by-launch episodes
                plan.set_tuning(tuning["row_tile"], tuning["chunk"], 0)
            plan.set_kernel_timing(True)
        plan.submit(0, I, S)
        plan.iterate(args.iters, cp.HIO, BETA)
        plan.assemble_volume(vol)
        if timed:
            c, cn, r, rn = plan.kernel_timing()
            col_ms += c; row_ms += r; col_n += cn; row_n += rn
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    for i in range(args.warmup):
        one_step(False)
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        lat.append(one_step(True))
        print(f"[bench] step {i + 1}/{args.steps}: {lat[-1] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    ms_per_step = total / args.steps * 1e3
    value = args.iters * NP * args.steps / total

    tr = load_traffic() if not args.amp16 else None
    roofline, iter_ms = roofline_of(col_ms, col_n, row_ms, row_n, args.iters * args.steps,
                                    amp_bytes=4 if args.amp16 else 8, traffic=tr)
    out = {
        "metric": "pattern-iterations/s at N=512,N_p=360 + p99 last-frame-to-volume latency",
        "value": round(value, 1),
        "unit": "pattern-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" + ("+f16amp" if args.amp16 else ""),
        "data": "synthetic",
        "config": {"workload": "cell-like 512^3 object, N=512, N_p=360, 200 HIO iterations "
                               "(beta 0.9, carousel every 10), prep + init + step D, one scan per step",
                   "N": N, "N_p": NP, "iterations": args.iters, "n_ei": N_EI},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)) * 1e3, 2),
                       "p99": round(float(np.percentile(lat, 99)) * 1e3, 2),
                       "what": "submit-to-volume time of a whole scan handed over at once (serving leg skipped)"},
        "iteration_only": {"ms_per_iteration": round(iter_ms, 4),
                           "pattern_iterations_per_s": round(NP / (iter_ms * 1e-3), 1)},
        "roofline": roofline,
        "tuning": tuning,
    }
    if not args.amp16 and args.iters == ITERS:
        print("[bench] FP16 amplitudes, error history", file=sys.stderr, flush=True)
        out["fp16_amplitudes"] = fp16_leg(cp, torch, scan, I, S, vol, stream, args)
        out["error_history_cost"] = error_history_leg(cp, torch, scan, I, S, stream, iter_ms)
    if not args.no_compare and args.iters == ITERS and not args.amp16:
        print("[bench] plain per-angle comparison", file=sys.stderr, flush=True)
        out["vs_plain_per_angle"] = plain_comparison(cp, torch, scan, I, S, args, iter_ms, quality_of())
    if not args.no_compare and args.iters == ITERS and not args.amp16:
        print("[bench] algorithm variants", file=sys.stderr, flush=True)
        out["variants"] = variants(cp, torch, scan, I, S, args)
    if args.guesses > 0 and args.iters == ITERS and not args.amp16:
        print(f"[bench] paper schedule, {args.guesses} guesses", file=sys.stderr, flush=True)
        out["paper_schedule"] = paper_schedule(cp, torch, scan, I, S, args, quality_of())
    if args.batch_scans > 0 and args.iters == ITERS and not args.amp16:
        print(f"[bench] batched: {args.batch_scans} scans of uneven size", file=sys.stderr, flush=True)
        out["batched_uneven_scans"] = batched_scans(cp, torch, scan, args, src_cache)
    if args.serve_scans > 0:
        out["latency_ms"] = serving_latency(cp, torch, scan, I, S, args, src_cache)
        out["latency_ms"]["whole_scan_p50"] = round(float(np.percentile(lat, 50)) * 1e3, 2)
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(scan)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
