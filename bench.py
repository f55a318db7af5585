"""Throughput of the polyspectrum estimator on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp16x2s|bf16x3|fp32]

Workload: one channel, 2^28 float32 samples of an AR(2) process (poles
0.95 e^{+-0.3 pi j}) driven by centred chi-square(1) noise, frame length
N = 8192, acG window (sigma_t = 0.14), N_f = 2048 frequencies, m = 10
frames per chunk (3276 chunks); S2, S3 and S4 with FP64 chunk averages and
error bars.  One step = one ps_execute over the whole resident record, by
default in the scaled FP16 x 2 precision (matrix-core S4 on operands the
centring pass splits).

Prints ONE JSON line (rank 0).  `value` is input samples per second.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N_SAMPLES = 1 << 28
N, NF, M = 8192, 2048, 10
SEED = 3
WORKLOAD = "ar2-chi2 1ch 2^28 f32, N=8192, N_f=2048, m=10, acG 0.14, S2+S3+S4"

# Calibrated HBM bytes of the S3 kernel at this workload (rocprofv3 FETCH_SIZE /
# WRITE_SIZE); reported as roofline.traffic only while the kernel's source is
# the one the counters were taken on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_s3_ar2_2p28_n8192_nf2048_traffic.json")

PEAK_HBM_GBS = 8000.0
# FP32 FMA on the vector ALUs: the vendor's 157.3 TFLOP/s (256 CUs x 128
# lanes x 2 flop x 2.4 GHz).  It does not need packed-FP32 instructions (which
# the library's device code is compiled without): a wave64 v_fma_f32 issues
# every 2.2-2.5 SIMD cycles with four or more waves per SIMD (measured on this
# chip; one wave alone issues every ~6 cycles).
PEAK_FP32_VALU_TFLOPS = 157.3


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def s3_flops_per_launch(n_frames: int, nf: int) -> float:
    """Algorithmic work of the S3 moment sums: one complex triple product
    a_k a_l conj(a_{k+l}) accumulated per frame and grid point k <= l
    (14 flops: 2 mul + 6 FMA)."""
    return 14.0 * (nf * (nf + 1) / 2) * n_frames


def s3_traffic():
    """Stored S3 HBM bytes per launch, or None when absent or stale."""
    try:
        from paper_2505_01231_amd.profile_summary import s3_source_digest
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        if t.get("source_sha256") != s3_source_digest():
            log("stored S3 traffic counters are stale (kernel source changed): traffic = null")
            return None
        return t["hbm_read_bytes_per_launch"] + t["hbm_write_bytes_per_launch"]
    except (OSError, ValueError, KeyError, RuntimeError):
        return None


def _oracle_chunks(args):
    """One worker of the multi-core CPU baseline: the oracle on chunks
    [c0, c1) of the record, returning every chunk's normalised spectra."""
    import numpy as np

    import oracle as O
    z, estimator = args
    out = O.polyspectra(np.asarray(z, dtype=np.float64), N, NF, M, window_kind="acg",
                        estimator=estimator, return_chunks=True)
    return out["chunks2"], out["chunks3"], out["chunks4"]


def _blas_info():
    try:
        from threadpoolctl import threadpool_info
        return [f"{d.get('internal_api')} {d.get('version')} ({d.get('num_threads')} threads)"
                for d in threadpool_info()]
    except Exception:  # pragma: no cover
        return []


def cpu_baseline(z, estimator="kstat", workers=None):
    """The FP64 oracle on bounded samples of the same workload (whole chunks
    of the record's start):
      * single-threaded: the oracle on the first chunks (its numpy kernels run
        on one core), sized to ~10 s;
      * all cores: the same oracle on one chunk per task over a process pool
        of min(16, cpu_count) workers (chunks are independent), ~10 s;
      * the factorized fourth-order form (Appendix H), single-threaded.
    Returns (record for the JSON line, oracle spectra of the single-thread
    sample for the accuracy check)."""
    import multiprocessing as mp

    import numpy as np

    import oracle as O
    chunk = N * M
    z64 = np.asarray(z[: chunk * 64], dtype=np.float64)
    t0 = time.perf_counter()
    O.polyspectra(z64[:chunk], N, NF, M, window_kind="acg", estimator=estimator)
    t1 = time.perf_counter() - t0
    n1 = int(max(1, min(6, 10.0 / max(t1, 1e-3))))
    t0 = time.perf_counter()
    ref = O.polyspectra(z64[: chunk * n1], N, NF, M, window_kind="acg", estimator=estimator)
    t1 = time.perf_counter() - t0
    single = chunk * n1 / t1

    cores = os.cpu_count() or 1
    workers = workers or max(1, min(16, cores))
    # whole rounds of one chunk per worker, ~10 s
    n_par = workers * int(max(1, min(4, round(10.0 / max(t1 / n1, 1e-3)))))
    # fresh worker interpreters (no inherited GPU state), one BLAS thread each
    ctx = mp.get_context("spawn")
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    os.environ.update({k: "1" for k in saved})
    try:
        with ctx.Pool(workers) as pool:
            pool.map(_oracle_chunks, [(z64[:chunk], estimator)] * workers)      # start-up and imports
            t0 = time.perf_counter()
            parts = pool.map(_oracle_chunks, [(z64[c * chunk:(c + 1) * chunk], estimator) for c in range(n_par)])
            tp = time.perf_counter() - t0
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    multi = chunk * n_par / tp

    t0 = time.perf_counter()
    O.polyspectra(z64[:chunk], N, NF, M, window_kind="acg", estimator="factorized")
    tf = time.perf_counter() - t0
    record = {
        "value": multi,
        "unit": "samples/s",
        "cores": workers,
        "kind": "oracle",
        "sample": f"{n_par} chunks ({chunk * n_par} samples) of the record's start, one chunk per task on "
                  f"{workers} worker processes (one thread each), full N_f=2048 grid, numpy float64, "
                  f"{tp:.1f} s",
        "host_cpu_count": cores,
        "single_thread": {"value": single, "chunks": n1, "seconds": round(t1, 2)},
        "factorized_single_thread": {"value": chunk / tf, "chunks": 1, "seconds": round(tf, 2),
                                     "form": "Appendix H centred c4 (S2, S3 unchanged)"},
        "numpy": np.__version__,
        "blas": _blas_info(),
        "extrapolated_seconds_for_2p28": N_SAMPLES / multi,
    }
    del parts
    return record, ref, n1


def accuracy(torch, dev, plan, z, ref, n_chunks):
    """Per-spectrum max relative error of the timed path against the FP64
    oracle on the same chunks: max |S_gpu - S_oracle| / max |S_oracle| over the
    whole grid, for S2, S3, S4 and their error bars."""
    import numpy as np
    x = torch.from_numpy(np.ascontiguousarray(z[: N * M * n_chunks])).to(dev)
    out = plan.execute(x)
    torch.cuda.synchronize()
    err = {}
    for k in ("s2", "s3", "s4"):
        got = torch.view_as_complex(getattr(out, k)).cpu().numpy()[0]
        want = ref[k][0]
        err[k] = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
        ge, we = getattr(out, k + "_err").cpu().numpy()[0], ref[k + "_err"][0]
        err[k + "_err"] = float(np.nanmax(np.abs(ge - we)) / np.nanmax(np.abs(we)))
    return {"max_rel_err": err, "chunks": n_chunks, "tolerance": 1e-5,
            "within_tolerance": all(v <= 1e-5 for v in err.values()),
            "note": "same plan (precision, estimator) as the timed steps, run on the chunks the CPU "
                    "baseline's single-thread oracle evaluated; normalised to each array's max |oracle|"}


def _gen_record(args):
    from paper_2505_01231_amd import synth
    n, seed = args
    z, clipped = synth.mixed_channels(int(n), seed=seed)
    return z, clipped


def run_batching(torch, dev, precision, n_records=256, out_budget=32e9, workers=16):
    """Batching form: 256 four-channel int16 records of uneven length
    (2^16..2^22 samples), each at a frame length drawn from {1024, 2048, 4096}
    with N_f = N/4, every combination orbit (10 / 40 / 76).  One plan holds the
    three frame lengths; records are taken in groups whose FP64 outputs fit
    `out_budget` bytes, and each group is ONE ps_execute mixing all frame
    lengths (every stage one launch over records x combinations).  The records
    are generated on a pool of worker processes."""
    import multiprocessing as mp

    import numpy as np

    from paper_2505_01231_amd import Plan, synth
    lengths = synth.uneven_record_lengths(n_records, seed=4)
    rng = np.random.default_rng(44)
    fls = [int(v) for v in rng.choice([1024, 2048, 4096], size=n_records)]
    t0 = time.perf_counter()
    jobs = [(int(L), 1000 + i) for i, L in enumerate(lengths)]
    if workers > 1:
        with mp.get_context("spawn").Pool(max(1, min(workers, os.cpu_count() or 1))) as pool:
            data = pool.map(_gen_record, jobs, chunksize=4)
    else:
        data = [_gen_record(j) for j in jobs]
    gen_s = time.perf_counter() - t0
    clipped = sum(c for _, c in data)
    xs = [torch.from_numpy(z).to(dev) for z, _ in data]
    del data
    torch.cuda.synchronize()
    log(f"batching: {n_records} records generated in {gen_s:.1f} s, {sum(int(x.shape[1]) for x in xs):,} samples "
        f"per channel, {clipped} clipped")
    with Plan(frame_len=1024, n_freq=256, m=10, window="acg", n_channels=4, precision=precision,
              frame_lens=(2048, 4096)) as p:
        n2, n3, n4 = len(p.combos2), len(p.combos3), len(p.combos4)
        nf = {n: p.frame_info(n)["n_freq"] for n in (1024, 2048, 4096)}
        out_bytes = {n: (n2 * nf[n] + (n3 + n4) * nf[n] ** 2) * 2 * 16 for n in nf}
        groups, cur, cur_b = [], [], 0
        for i in range(n_records):
            if cur and cur_b + out_bytes[fls[i]] > out_budget:
                groups.append(cur)
                cur, cur_b = [], 0
            cur.append(i)
            cur_b += out_bytes[fls[i]]
        groups.append(cur)
        ws_bytes = max(p.workspace_bytes([xs[i] for i in g], frame_lens=[fls[i] for i in g]) for g in groups)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
        # output sets per frame length for the most records of that length in a group, reused by every group
        need = {n: max(sum(1 for i in g if fls[i] == n) for g in groups) for n in nf}
        outs_by_n = {n: [p.allocate_outputs(dev, n) for _ in range(need[n])] for n in nf}

        def outs_of(g):
            used = {n: 0 for n in nf}
            res = []
            for i in g:
                res.append(outs_by_n[fls[i]][used[fls[i]]])
                used[fls[i]] += 1
            return res

        g0 = groups[0]
        tune = p.autotune([xs[i] for i in g0], reps=1, workspace=ws, outputs=outs_of(g0),
                          frame_lens=[fls[i] for i in g0])       # also the warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for g in groups:
            p.execute([xs[i] for i in g], workspace=ws, outputs=outs_of(g), frame_lens=[fls[i] for i in g])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    ns = sum(int(x.shape[1]) * 4 for x in xs)
    per_n = {str(n): {"records": fls.count(n), "n_freq": nf[n]} for n in nf}
    log(f"batching: {ns / dt:.3e} channel-samples/s over {len(groups)} executes")
    del ws, outs_by_n, xs
    return {"records": n_records, "channels": 4, "precision": precision, "combinations": [n2, n3, n4],
            "executes": len(groups),
            "frame_lengths_per_execute": "1024, 2048 and 4096 mixed", "channel_samples": ns, "seconds": dt,
            "channel_samples_per_s": ns / dt, "per_frame_length": per_n, "workspace_bytes": ws_bytes,
            "tuning": tune["best"], "generation_s": gen_s,
            "note": "each ps_execute runs every stage as one launch over its records (all three frame lengths) x "
                    "combinations; records grouped so that each execute's FP64 outputs stay under "
                    f"{out_budget / 1e9:.0f} GB; tile order chosen by ps_plan_autotune on the first group"}


def run_streaming(torch, dev, precision, stream_samples=10**10, pool=16, per_push=16, depth=3):
    """Streaming form: consecutive 2^20-sample windows of an amplitude-ramped
    AR(2)/chi-square stream, pushed from pinned host buffers through
    ps_streamer, `per_push` consecutive windows per push (H2D copies overlap
    computation; every window gets its own spectra), until at least
    `stream_samples` samples have been processed (the whole 10^10-sample
    stream by default).  A pool of `pool` generated windows is reused
    cyclically, so the stream's content repeats every `pool` windows."""
    from paper_2505_01231_amd import Plan, Streamer, synth
    W = 1 << 20
    n_windows = -(-stream_samples // (W * per_push)) * per_push
    pool_host = torch.empty(pool * W, dtype=torch.float32, pin_memory=True)
    pool_host.copy_(torch.from_numpy(synth.modulated_ar2(pool * W, seed=5, start=0, total=W * pool)))
    groups = [pool_host[(g * per_push) % pool * W:((g * per_push) % pool + per_push) * W]
              for g in range(pool // per_push)]
    with Plan(frame_len=4096, n_freq=1024, m=10, window="acg", precision=precision) as p:
        st = Streamer(p, W, dtype=torch.float32, depth=depth, windows_per_push=per_push)
        outs = [[p.allocate_outputs(dev) for _ in range(per_push)] for _ in range(depth)]
        slots = [st.push(groups[g % len(groups)], outs[g]) for g in range(depth)]   # warm-up
        for sl in slots:
            st.wait(sl)
        torch.cuda.synchronize()
        n_push = n_windows // per_push
        t0 = time.perf_counter()
        slots = []
        for g in range(n_push):
            if g >= depth:
                st.wait(slots[g - depth])
            slots.append(st.push(groups[g % len(groups)], outs[g % depth]))
        for sl in slots[-depth:]:
            st.wait(sl)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st.close()
        total = W * per_push * n_push
    rate = total / dt
    # reference: a plain pinned host-to-device copy of the same volume
    big = torch.empty(W * 16, dtype=torch.float32, pin_memory=True)
    dst = torch.empty(W * 16, dtype=torch.float32, device=dev)
    dst.copy_(big, non_blocking=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(4):
        dst.copy_(big, non_blocking=True)
    torch.cuda.synchronize()
    link = 4 * big.numel() * 4 / (time.perf_counter() - t0) / 1e9
    log(f"streaming {rate:.3e} samples/s, H2D {total * 4 / dt / 1e9:.1f} GB/s (plain pinned copy {link:.1f} GB/s)")
    return {"windows": total // W, "window_samples": W, "samples_per_s": rate,
            "h2d_GBps": total * 4 / dt / 1e9, "plain_pinned_h2d_GBps": link, "seconds": dt,
            "stream_samples": total, "windows_per_push": per_push,
            "note": f"N=4096, N_f=1024, m=10, {per_push} windows per push, depth-{depth} pinned ring; every "
                    f"window of the {total:,}-sample stream is copied and transformed (a pool of {pool} "
                    "generated windows cycled); the H2D rate includes the copy/compute overlap"}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp16x2s", choices=("fp32", "bf16x3", "fp16x2s"))
    ap.add_argument("--fp32-steps", type=int, default=3,
                    help="timed steps of the batched all-FP32 path (for mixed-vs-FP32)")
    ap.add_argument("--plain-steps", type=int, default=1, help="timed steps of the per-chunk FP32 path")
    ap.add_argument("--interlaced-steps", type=int, default=2,
                    help="timed steps of the interlaced form (second frame set shifted by N/2, "
                         "spectra averaged) on the same record")
    ap.add_argument("--sequential-steps", type=int, default=1,
                    help="timed steps of sequential spectra (every chunk's estimate kept) over the first "
                         "2^22 samples at N = 1024, N_f = 256")
    ap.add_argument("--estimator", default="kstat", choices=("kstat", "c3opt"),
                    help="estimator of the main leg (c3opt: S3 by c3^(opt), one more row per chunk in S3)")
    ap.add_argument("--c3opt-steps", type=int, default=2,
                    help="timed steps with S3 by the c3^(opt) estimator (one extra mean row per chunk) "
                         "on the same record")
    ap.add_argument("--graph-steps", type=int, default=5,
                    help="timed replays of the main step captured as one HIP graph")
    ap.add_argument("--direct-steps", type=int, default=2,
                    help="timed steps of a frame length that is not a power of two (N = 1536, the direct "
                         "transform) on the first 2^24 samples, S2+S3+S4")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batching", action="store_true",
                    help="skip the batching form (four-channel int16 records of uneven length "
                         "(2^16..2^22), N in {1024, 2048, 4096}, N_f = N/4, every combination orbit)")
    ap.add_argument("--batching-records", type=int, default=256,
                    help="records of the batching form (the first ones of the same seeded set)")
    ap.add_argument("--gen-workers", type=int, default=16,
                    help="worker processes generating the batching records (1: in this process, "
                         "e.g. under a profiler that attaches to every process)")
    ap.add_argument("--no-streaming", action="store_true",
                    help="skip the streaming form (the 10^10-sample stream in windows of 2^20 samples "
                         "from pinned host memory, 16 windows per push, N = 4096, N_f = 1024, "
                         "copy/compute overlap)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain elementwise copy of 1 GiB (3 launches) so that profiler "
                         "byte counters can be scaled against a kernel of known traffic")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        msg = (f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
               "(the estimator shards chunks across GPUs without exchange until one final "
               "all-reduce; that path is not built here)")
        print(msg, file=sys.stderr)
        print(json.dumps({"error": msg, "n_gpus": args.gpus}))
        return 2

    import numpy as np
    import torch

    from paper_2505_01231_amd import Plan, synth

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)          # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del a, b
        log("copy calibration: 3 x (1 GiB read + 1 GiB write)")
    log("generating input")
    z = synth.ar2_chi2(N_SAMPLES, seed=SEED)
    x = torch.from_numpy(z).to(dev)
    torch.cuda.synchronize()

    plan = Plan(frame_len=N, n_freq=NF, m=M, window="acg", precision=args.precision, estimator=args.estimator)
    n_chunks, _ = plan.record_info(N_SAMPLES)
    n_frames = n_chunks * M
    # rows the S3 kernel sums per launch (c3^(opt): m shifted frames + one mean row per chunk)
    s3_rows = n_chunks * (M + 1) if args.estimator == "c3opt" else n_frames
    ws = torch.empty(plan.workspace_bytes([x]), dtype=torch.uint8, device=dev)
    outs = [plan.allocate_outputs(dev)]
    log(f"workspace {ws.numel() / 2**30:.2f} GiB, chunks {n_chunks}")

    for i in range(args.warmup):
        plan.execute([x], workspace=ws, outputs=outs)
    torch.cuda.synchronize()
    log("warmup done")

    plan.profile(True)
    plan.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        plan.execute([x], workspace=ws, outputs=outs)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stages = plan.profile_read()
    plan.profile(False)
    log(f"timed {args.steps} steps in {elapsed:.3f} s")

    value = N_SAMPLES * args.steps / elapsed
    s3_ms, s3_n = stages["s3"]
    s3_avg_ms = s3_ms / max(1, s3_n)
    achieved = s3_flops_per_launch(s3_rows, NF) / (s3_avg_ms * 1e-3) / 1e12
    stage_ms = {k: round(v[0] / max(1, args.steps), 4) for k, v in stages.items()}

    # The same step replayed from one captured HIP graph (ps_graph_create /
    # ps_graph_launch) on the same workspace and outputs.
    graph = None
    if args.graph_steps > 0:
        g = plan.graph([x], workspace=ws, outputs=outs)
        g.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.graph_steps):
            g.launch()
        torch.cuda.synchronize()
        dt_g = time.perf_counter() - t0
        g.close()
        graph = {"samples_per_s": N_SAMPLES * args.graph_steps / dt_g, "ms_per_step": dt_g / args.graph_steps * 1e3,
                 "steps": args.graph_steps}
        log(f"graph replay {graph['samples_per_s']:.3e} samples/s")

    # The plain FP32 path: same kernels, one chunk per launch (the paper's structure).
    plain = None
    if args.plain_steps > 0:
        with Plan(frame_len=N, n_freq=NF, m=M, window="acg", precision="fp32", schedule="per_chunk") as pp:
            wsp = torch.empty(pp.workspace_bytes([x]), dtype=torch.uint8, device=dev)
            op = [pp.allocate_outputs(dev)]
            pp.execute([x], workspace=wsp, outputs=op)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.plain_steps):
                pp.execute([x], workspace=wsp, outputs=op)
            torch.cuda.synchronize()
            plain = N_SAMPLES * args.plain_steps / (time.perf_counter() - t0)
        log(f"plain per-chunk path {plain:.3e} samples/s")
    batched_fp32 = value if args.precision == "fp32" else None
    if batched_fp32 is None and args.fp32_steps > 0:
        with Plan(frame_len=N, n_freq=NF, m=M, window="acg", precision="fp32") as pf:
            wsf = torch.empty(pf.workspace_bytes([x]), dtype=torch.uint8, device=dev)
            of = [pf.allocate_outputs(dev)]
            pf.execute([x], workspace=wsf, outputs=of)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.fp32_steps):
                pf.execute([x], workspace=wsf, outputs=of)
            torch.cuda.synchronize()
            batched_fp32 = N_SAMPLES * args.fp32_steps / (time.perf_counter() - t0)
            del wsf, of
        log(f"batched fp32 path {batched_fp32:.3e} samples/s")

    # S4 on the matrix cores: executed and useful work of one launch.
    s4_ms, s4_n = stages["s4"]
    s4_avg_ms = s4_ms / max(1, s4_n)
    n_tiles = (NF // 64) * (NF // 64 + 1) // 2
    s4_info = {"avg_launch_ms": s4_avg_ms,
               "useful_tflops": 10.0 * (NF * (NF + 1) / 2) * n_frames / (s4_avg_ms * 1e-3) / 1e12}
    if args.precision != "fp32":
        if args.precision == "bf16x3":
            # per 64 x 64 tile and chunk: 4 waves x 4 K steps x 5 sums MFMA 32x32x16
            mfma_flops = n_tiles * n_chunks * 4 * 20 * (32 * 32 * 16 * 2)
        else:
            # operands split by the centring pass (m <= 10): per 64 x 64 tile
            # and chunk 4 waves x 2 K steps x 5 sums MFMA 32x32x16 (f16)
            mfma_flops = n_tiles * n_chunks * 4 * 10 * (32 * 32 * 16 * 2)
        s4_info.update({"mfma_executed_tflops": mfma_flops / (s4_avg_ms * 1e-3) / 1e12,
                        "mfma_peak_tflops": 2500.0,
                        "mfma_frac_of_peak": mfma_flops / (s4_avg_ms * 1e-3) / 2.5e15})
        if args.precision == "fp16x2s":
            # Upper bound on the matrix pipe's busy fraction set by the FP64
            # combination: per wave and chunk the compiled kernel issues 10
            # MFMA 32x32x16 (32 cycles each), 129 FP64-rate and 81 other vector
            # instructions; at two waves per SIMD these cost 5.27 and 3.18 SIMD
            # cycles each (vector-issue timing kernel), and at best one wave's
            # matrix work hides under the other's vector work.
            valu_cycles = 129 * 5.27 + 81 * 3.18
            s4_info["mfma_ceiling_frac"] = round(10 * 32 / valu_cycles, 3)
            s4_info["mfma_ceiling_basis"] = ("FP64 k-statistic combination: 16 points x 8 FP64-rate "
                                             "instructions per wave and chunk against 10 MFMA 32x32x16")

    # Interlaced windows: the same record with a second frame set shifted by N/2
    # (twice the frames), spectra of both sets averaged.
    interlaced = None
    if args.interlaced_steps > 0:
        with Plan(frame_len=N, n_freq=NF, m=M, window="acg", precision=args.precision, interlaced=True) as pi:
            wsi = torch.empty(pi.workspace_bytes([x]), dtype=torch.uint8, device=dev)
            oi = [pi.allocate_outputs(dev)]
            pi.execute([x], workspace=wsi, outputs=oi)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.interlaced_steps):
                pi.execute([x], workspace=wsi, outputs=oi)
            torch.cuda.synchronize()
            dt_i = time.perf_counter() - t0
            interlaced = {"samples_per_s": N_SAMPLES * args.interlaced_steps / dt_i,
                          "ms_per_step": dt_i / args.interlaced_steps * 1e3,
                          "frames_per_step": 2 * n_frames, "steps": args.interlaced_steps}
            del wsi, oi
        log(f"interlaced {interlaced['samples_per_s']:.3e} samples/s")

    # c3^(opt) for S3: the centring pass also writes m shifted frames and a
    # mean row per chunk, S3 sums m + 1 rows; S2 and S4 unchanged.
    c3opt = None
    if args.c3opt_steps > 0:
        with Plan(frame_len=N, n_freq=NF, m=M, window="acg", precision=args.precision, estimator="c3opt") as po:
            wso = torch.empty(po.workspace_bytes([x]), dtype=torch.uint8, device=dev)
            oo = [po.allocate_outputs(dev)]
            po.execute([x], workspace=wso, outputs=oo)
            torch.cuda.synchronize()
            po.profile(True)
            po.profile_read()
            t0 = time.perf_counter()
            for _ in range(args.c3opt_steps):
                po.execute([x], workspace=wso, outputs=oo)
            torch.cuda.synchronize()
            dt_o = time.perf_counter() - t0
            st_o = po.profile_read()
            po.profile(False)
            c3opt = {"samples_per_s": N_SAMPLES * args.c3opt_steps / dt_o,
                     "ms_per_step": dt_o / args.c3opt_steps * 1e3, "steps": args.c3opt_steps,
                     "workspace_bytes": int(wso.numel()),
                     "stage_ms_per_step": {k: round(v[0] / args.c3opt_steps, 4) for k, v in st_o.items()}}
            del wso, oo
        log(f"c3opt {c3opt['samples_per_s']:.3e} samples/s")

    # A frame length that is not a power of two (the direct transform of the
    # frames in FP64 instead of the FFT), the whole estimator on a prefix.
    direct = None
    if args.direct_steps > 0:
        n_d, N_d = 1 << 24, 1536
        xd = x[:n_d]
        with Plan(frame_len=N_d, n_freq=N_d // 4 + 1, m=M, window="acg", precision=args.precision) as pd:
            wsd = torch.empty(pd.workspace_bytes([xd]), dtype=torch.uint8, device=dev)
            od = [pd.allocate_outputs(dev)]
            pd.execute([xd], workspace=wsd, outputs=od)
            torch.cuda.synchronize()
            pd.profile(True)
            pd.profile_read()
            t0 = time.perf_counter()
            for _ in range(args.direct_steps):
                pd.execute([xd], workspace=wsd, outputs=od)
            torch.cuda.synchronize()
            dt_d = time.perf_counter() - t0
            st_d = pd.profile_read()
            pd.profile(False)
            direct = {"frame_len": N_d, "n_freq": N_d // 4 + 1, "samples": n_d,
                      "samples_per_s": n_d * args.direct_steps / dt_d,
                      "ms_per_step": dt_d / args.direct_steps * 1e3, "steps": args.direct_steps,
                      "stage_ms_per_step": {k: round(v[0] / args.direct_steps, 4) for k, v in st_d.items()}}
            del wsd, od
        log(f"direct transform (N = 1536) {direct['samples_per_s']:.3e} samples/s")

    # Sequential spectra: each chunk's short-time estimate written out (FP64
    # S2, S3, S4 and error-bar arrays per chunk), on a prefix of the record.
    sequential = None
    if args.sequential_steps > 0:
        n_seq, n_s, nf_s = 1 << 22, 1024, 256
        xs_ = x[:n_seq]
        with Plan(frame_len=n_s, n_freq=nf_s, m=M, window="acg", precision=args.precision) as ps_:
            out_ = ps_.sequential(xs_)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.sequential_steps):
                out_ = ps_.sequential(xs_, workspace=ps_._last_workspace)
            torch.cuda.synchronize()
            dt_s = time.perf_counter() - t0
            sequential = {"chunks_per_s": out_.n_chunks * args.sequential_steps / dt_s,
                          "samples_per_s": n_seq * args.sequential_steps / dt_s,
                          "ms_per_step": dt_s / args.sequential_steps * 1e3, "chunks": out_.n_chunks,
                          "frame_len": n_s, "n_freq": nf_s,
                          "output_bytes_per_step": sum(t.numel() * 8 for t in (out_.s2, out_.s2_err, out_.s3,
                                                                                out_.s3_err, out_.s4, out_.s4_err))}
            del out_
        log(f"sequential {sequential['chunks_per_s']:.3e} chunks/s")

    # (the four-channel records are mostly cross-channel S4, which has a
    # matrix-core kernel in BF16 x 3 only)
    batching = None if args.no_batching else run_batching(torch, dev, "fp32" if args.precision == "fp32" else "bf16x3",
                                                          n_records=args.batching_records,
                                                          workers=args.gen_workers)
    streaming = None if args.no_streaming else run_streaming(torch, dev, args.precision)

    cpu, acc = None, None
    if not args.no_cpu_baseline:
        cpu, ref, n_ref = cpu_baseline(z, estimator=args.estimator)
        log(f"cpu baseline {cpu['value']:.3e} samples/s on {cpu['cores']} workers "
            f"(single thread {cpu['single_thread']['value']:.3e})")
        acc = accuracy(torch, dev, plan, z, ref, n_ref)
        log(f"accuracy vs oracle: {acc['max_rel_err']}")

    # Achieved HBM rates of the bandwidth-bound stages from their algorithmic
    # bytes per step: the FFT reads the samples of every full chunk and writes
    # K = 2 N_f - 1 complex FP32 coefficients per frame; the centring reads and
    # writes every coefficient and, for the scaled FP16 x 2 S4, writes each
    # chunk's operand records (3 values x 3 16-byte pieces and one 16-byte
    # (p, s^2) pair per column, N_f padded to 64 columns); S2 reads the first
    # N_f columns.
    K_COEF = 2 * NF - 1
    rec_cols = (NF + 63) // 64 * 64
    # (c3^(opt): the centring also writes the S3 rows, m + 1 per chunk)
    alg_bytes = {"fft": 4 * n_frames * N + 8 * K_COEF * n_frames,
                 "mean": 16 * K_COEF * n_frames + (8 * K_COEF * s3_rows if args.estimator == "c3opt" else 0)
                 + (160 * rec_cols * n_chunks if args.precision == "fp16x2s" else 0),
                 "s2": 8 * NF * n_frames}
    stage_rates = {f"{k}_hbm_gbps": (b / (stage_ms[k] * 1e-3) / 1e9 if stage_ms.get(k) else None)
                   for k, b in alg_bytes.items()}
    stage_rates.update({"algorithmic_bytes_per_step": alg_bytes, "hbm_peak_gbps": 8000.0})
    # S3 is bound by the vector ALUs; its HBM rate from the stored counters
    # (L2-miss bytes per launch) and from its algorithmic bytes (the
    # coefficient region read once)
    s3_tr = s3_traffic() if args.estimator == "kstat" else None
    stage_rates["s3_hbm_gbps_counters"] = s3_tr / (s3_avg_ms * 1e-3) / 1e9 if s3_tr else None
    stage_rates["s3_hbm_gbps_algorithmic"] = 8 * K_COEF * n_frames / (s3_avg_ms * 1e-3) / 1e9

    line = {
        "metric": "input samples/sec for S2+S3+S4 at N_f=2048; mixed vs FP32 at <=1e-5 rel err; MFMA%",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else args.precision,
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "precision": args.precision, "estimator": args.estimator,
                   "n_chunks": n_chunks,
                   "samples_per_step": N_SAMPLES},
        "roofline": {
            "kernel": "k_s3 (S3 triple-product moment sums)",
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_VALU_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_VALU_TFLOPS,
            "peak_note": "vendor FP32 vector figure; reachable without packed FP32 (a wave64 v_fma_f32 "
                         "issues every 2.2-2.5 SIMD cycles at >= 4 waves per SIMD, measured)",
            "traffic": s3_traffic() if args.estimator == "kstat" else None,
            "avg_launch_ms": s3_avg_ms,
            "flops_per_launch": s3_flops_per_launch(s3_rows, NF),
        },
        "cpu_baseline": cpu,
        "accuracy": acc,
        "paths": {"main": args.precision, "main_value": value, "batched_fp32": batched_fp32,
                  "per_chunk_fp32": plain,
                  "speedup_vs_batched_fp32": (value / batched_fp32) if batched_fp32 else None,
                  "speedup_vs_per_chunk_fp32": (value / plain) if plain else None},
        "graph": graph,
        "s4_matrix_cores": s4_info,
        "interlaced": interlaced,
        "c3opt": c3opt,
        "direct_transform": direct,
        "sequential": sequential,
        "batching": batching,
        "streaming": streaming,
        "stage_ms_per_step": stage_ms,
        "stage_rates": stage_rates,
    }
    print(json.dumps(line), flush=True)
    plan.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
