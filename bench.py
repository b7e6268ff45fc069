"""Benchmark: TT rounding of X = A + B (N=16, I=262144, A and B random TTs of
rank 20, formal ranks 40, ~47 GB of FP64 cores) at relative tolerance 1e-8 on
one MI355X.

One step = the whole path for this workload on inputs resident in HBM:
ttr_add(A, B) -> X, then ttr_round(X) (orthonormalization sweep, norm and
threshold, truncation sweep).  `value` is the rounding's core-GB/s = bytes of
X's cores per second of ttr_round time (HIP events around the call inside each
step); `ms_per_step` is the whole step.  The JSON line also carries the
dominant kernel's roofline position (measured with HIP events on the library's
stream during the timed steps) and the FP64 CPU oracle timed on a bounded
sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--I 262144]
"""

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6        # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
RIDGE = FP64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)   # flop/byte


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# the sources that define the streaming kernels whose counters
# profiles/pmc_traffic.json records, and the host code that launches them
TRAFFIC_SOURCES = ("ttr_api.hip", "ttr_host.h", "ttr_internal.h", "ttr_mfma.hip", "ttr_stream.hip")


def source_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2011_06532_amd", "csrc")
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_traffic(kernel_class, per_launch_bytes):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when it is absent or was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("source_hash") != source_hash():
        return None
    ent = d.get("kernels", {}).get(kernel_class)
    if not ent:
        return None
    return ent.get("hbm_bytes_per_launch")


def sample_entries(cores, R, I, idx):
    """Entries X(i_1, ..., i_N) at the rows of idx, as products of slices
    (the cores' slices are gathered on the device, multiplied on the host)."""
    import numpy as np
    S, N = idx.shape
    v = np.ones((S, 1))
    for n in range(N):
        r0, r1 = R[n], R[n + 1]
        t3 = cores[n][: r0 * I[n] * r1].view(r1, I[n], r0)      # [b][i][a]
        sl = t3[:, idx[:, n], :].permute(1, 2, 0).cpu().numpy()  # [s][a][b]
        v = np.einsum("sa,sab->sb", v, sl)
    return v[:, 0]


def error_bound_figures(h, torch, Y, tol):
    """Two device-side figures of ||X - X~|| / ||X|| for the last RLR rounding
    on the handle, against Alg. 2's guarantee (<= tol):
    * tail: sqrt(sum over links of the discarded singular values squared) /
      ||X|| -- the truncation steps' own sums (every discarded direction is
      orthogonal to the kept ones and to each other);
    * pythagoras: sqrt(||X||^2 - ||X~||^2) / ||X||, with ||X~|| = ||X~_N||_F
      because the output cores 1..N-1 are left-orthonormal.  The difference
      of two squared norms that agree to rounding leaves this figure a floor
      of about sqrt(8 N u) (~1e-7 at N = 16): below it, it only says "no
      larger than the floor".
    ||X|| is the norm the rounding computed for its threshold.  `within_tol`
    takes the tail figure, and the Pythagoras figure where it is above its
    floor."""
    st = h.round_stats()
    nrm = st["norm"]
    tail = math.sqrt(sum(st["tail2"])) / nrm if nrm > 0 else 0.0
    n_last = Y.R[-2] * Y.I[-1] * Y.R[-1]
    ny = float(torch.linalg.vector_norm(Y.cores[-1][:n_last]).item())
    pyth = math.sqrt(max(nrm * nrm - ny * ny, 0.0)) / nrm if nrm > 0 else 0.0
    floor = math.sqrt(8.0 * len(Y.I) * 2.0 ** -53)
    return {"tol": tol, "rel_err_tail": tail, "rel_err_pythagoras": pyth, "pythagoras_floor": floor,
            "within_tol": bool(tail <= tol and pyth <= max(tol * (1 + 1e-6), floor)),
            "jacobi_sweeps": st["sweeps"]}


def bench_batched(h, ttr, torch, steps, count=512, per_tensor=True):
    """512 independent Y + Y + 1e-9 E tensors (N=8, I_n log-uniform in
    [64, 4096], ranks 2r+2 with r uniform in 1..31), tol 1e-7: one replay of the
    batched graph against one ttr_round call per tensor."""
    import synth
    shapes = synth.batched_shapes(count)
    log(f"batched: generating {count} tensors")
    Xs = []
    for t, (I, r) in enumerate(shapes):
        Y = ttr.TT.from_numpy(synth.random_tt(3, t, "Y", I, r, scaled=True))
        E = ttr.TT.from_numpy(synth.random_tt(3, t, "E", I, [2] * 7, scaled=True, first_core_factor=1e-9))
        Xs.append(h.add(1.0, h.add(1.0, Y, 1.0, Y), 1.0, E))
    torch.cuda.synchronize()
    nbytes = sum(8 * X.R[n] * X.I[n] * X.R[n + 1] for X in Xs for n in range(X.N))
    expect = [[1] + list(r) + [1] for _, r in shapes]
    tol = synth.TOL[3]
    out = {"tensors": count, "core_bytes": nbytes}
    stream = torch.cuda.current_stream()
    for prec in ("fp64", "mixed"):
        log(f"batched {prec}: plan + autotune")
        Ys, ranks = h.round_batched(Xs, tol, prec, tune=True)
        torch.cuda.synchronize()
        plan = h.batch_plan()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            Ys, ranks = h.round_batched(Xs, tol, prec, outs=Ys, ranks=ranks)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        rk = ranks.cpu().tolist()
        res = {"ms_per_batch": round(ms, 3), "core_GBps": round(nbytes / (ms * 1e-3) / 1e9, 2),
               "ranks_ok": rk == expect, "spw_target": plan["spw_target"], "grid_cap": plan["grid_cap"],
               "graph_nodes": plan["graph_nodes"],
               "autotune": [[c["spw"], c["grid"], round(c["ms"], 3)] for c in plan["candidates"]]}
        out[prec] = res
        if not per_tensor:
            continue
        # one launch sequence per tensor (the single path, host-planned)
        log(f"batched {prec}: one ttr_round per tensor")
        outs1 = [ttr.TT.empty(X.I, [X.R[n] * X.I[n] * X.R[n + 1] for n in range(X.N)]) for X in Xs]
        for X, Y1 in zip(Xs, outs1):
            h.round(X, tol, "RLR", prec, out=Y1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        same = True
        for X, Y1, r in zip(Xs, outs1, expect):
            Y1 = h.round(X, tol, "RLR", prec, out=Y1)
            same = same and (Y1.R == r)
        torch.cuda.synchronize()
        ms1 = (time.perf_counter() - t0) * 1e3
        res["ms_one_launch_sequence_per_tensor"] = round(ms1, 3)
        res["speedup_vs_per_tensor"] = round(ms1 / ms, 2)
        res["per_tensor_ranks_ok"] = same
        out[prec] = res
    del Xs
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(I_sample, I_sample_1t=4096):
    """FP64 CPU oracle on bounded samples of the same workload (I reduced):
    the rounding alone (inputs in RAM), with the BLAS on all its threads and
    on one thread."""
    import oracle as O
    import synth
    from threadpoolctl import threadpool_info, threadpool_limits

    def timed(I_s):
        d = synth.sum_r40(I_override=I_s)
        X = O.add(1.0, d["A"], 1.0, d["B"])
        del d
        t0 = time.perf_counter()
        O.round_tt(X, synth.TOL[1], "RLR")
        return O.tt_bytes(X), time.perf_counter() - t0

    info = threadpool_info()
    threads = max([x.get("num_threads", 1) for x in info] or [1])
    blas = ", ".join(sorted({f"{x.get('internal_api', '?')} {x.get('version', '')}".strip() for x in info
                             if x.get("user_api") == "blas"})) or "unknown"
    nbytes, dt = timed(I_sample)
    with threadpool_limits(limits=1):
        nbytes1, dt1 = timed(I_sample_1t)
    return {
        "value": round(nbytes / dt / 1e9, 5),
        "unit": "GB/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": f"same workload with I={I_sample} instead of 262144 ({nbytes / 1e9:.3f} GB of cores), "
                  f"RLR round of X = A + B, NumPy FP64 on {blas}, {threads} threads, {dt:.2f} s",
        "ms_per_round": round(dt * 1e3, 2),
        "one_thread": {"value": round(nbytes1 / dt1 / 1e9, 5), "unit": "GB/s", "I": I_sample_1t,
                       "core_bytes": nbytes1, "ms_per_round": round(dt1 * 1e3, 2)},
        "cpu_model": cpu_model(),
        "nproc": os.cpu_count(),
    }


def copy_calibration(gib):
    """A plain copy of known size, for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = int(gib * (1 << 30)) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": n * 8, "copies": 3}), flush=True)


def bench_large(h, ttr, torch, steps):
    """Hadamard product of two random TTs (N=10, I=16384, ranks 16 with 2^-b
    rank weights) -> formal ranks 256 (68.7 GB of cores), then ttr_round at tol
    1e-6: the rank 65..256 path."""
    import synth
    torch.cuda.empty_cache()   # blocks cached by the earlier legs are returned to the device
    log("large: generating A, B (N=10, I=16384, ranks 16)")
    d = synth.hadamard_r256()
    A = ttr.TT.from_numpy(d["A"])
    B = ttr.TT.from_numpy(d["B"])
    tol = d["tol"]
    del d
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    X = h.hadamard(A, B)
    torch.cuda.synchronize()
    e0.record(stream)
    X = h.hadamard(A, B, out=X)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_had = e0.elapsed_time(e1)
    nbytes = sum(8 * X.R[n] * X.I[n] * X.R[n + 1] for n in range(X.N))
    out = {"workload": "A * B (Hadamard), N=10, I=16384, A,B random TTs of rank 16 with 2^-b rank weights, "
                       f"formal ranks 256, ttr_round tol {tol:g}",
           "core_bytes_X": nbytes, "ms_hadamard": round(ms_had, 3),
           "hadamard_GBps": round(nbytes / (ms_had * 1e-3) / 1e9, 1)}
    Y = None
    ranks64 = None
    for prec, direction in (("fp64", "RLR"), ("mixed", "RLR"), ("fp64", "LRL")):
        log(f"large: warm-up round {prec} {direction}")
        Y = h.round(X, tol, direction, prec, out=Y)
        torch.cuda.synchronize()
        ts = []
        for k in range(max(1, min(steps, 3)) if direction == "RLR" else 1):
            e0.record(stream)
            Y = h.round(X, tol, direction, prec, out=Y)
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
            log(f"large {prec} {direction}: round {k + 1}: {ts[-1]:.1f} ms")
        st = h.round_stats()
        ms = sum(ts) / len(ts)
        r = {"ms_per_round": round(ms, 3), "round_core_GBps": round(nbytes / (ms * 1e-3) / 1e9, 2),
             "rounds": len(ts), "ranks": list(Y.R), "gram_passes": st["gram_passes"]}
        if direction == "RLR":
            r["error_bound"] = error_bound_figures(h, torch, Y, tol)
        else:
            r["jacobi_sweeps"] = st["sweeps"]
        if ranks64 is None:
            ranks64 = list(Y.R)
        else:
            r["ranks_equal_fp64_rlr"] = list(Y.R) == ranks64
        out[f"{prec}_{direction}"] = r
    out["mixed_speedup"] = round(out["fp64_RLR"]["ms_per_round"] / out["mixed_RLR"]["ms_per_round"], 3)
    # the same rounding with the Hadamard product kept implicit (A * B never
    # formed, §3.2.2), FP64 RLR, against the formed path's ranks
    del X
    torch.cuda.empty_cache()
    log("large: implicit Hadamard rounding")
    Yi = h.round_hadamard(A, B, tol, "RLR", "fp64", out=Y)
    torch.cuda.synchronize()
    ts = []
    for k in range(max(1, min(steps, 3))):
        e0.record(stream)
        Yi = h.round_hadamard(A, B, tol, "RLR", "fp64", out=Y)
        e1.record(stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
        log(f"large implicit: round {k + 1}: {ts[-1]:.1f} ms")
    ms_i = sum(ts) / len(ts)
    out["implicit_hadamard_RLR"] = {"ms_per_round": round(ms_i, 3), "ranks": list(Yi.R),
                                    "ranks_equal_fp64_rlr": list(Yi.R) == ranks64,
                                    "error_bound": error_bound_figures(h, torch, Yi, tol),
                                    "speedup_vs_hadamard_then_round":
                                        round((out["fp64_RLR"]["ms_per_round"] + ms_had) / ms_i, 3)}
    X = None
    del X, Y, A, B
    torch.cuda.empty_cache()
    return out


def bench_norms(h, torch, X, size_x, steps):
    """The three norm methods of §3.2.4 on the same resident X: the inner
    product (gram), its symmetric form (sym) and orthonormalization (ortho)."""
    log("norm methods")
    stream = torch.cuda.current_stream()
    norms = {}
    for meth in ("gram", "sym", "ortho"):
        h.norm(X, meth)
        torch.cuda.synchronize()
        h.set_profiling(True)
        evn = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        vals = []
        for k in range(steps):
            evn[k][0].record(stream)
            vals.append(h.norm(X, meth))
            evn[k][1].record(stream)
        torch.cuda.synchronize()
        pn = h.profile()
        h.set_profiling(False)
        ms_n = sum(a.elapsed_time(b) for a, b in evn) / steps
        norms[meth] = {"ms": round(ms_n, 3), "core_GBps": round(size_x / (ms_n * 1e-3) / 1e9, 2),
                       "norm": vals[-1],
                       "kernel_ms": {c: round(pn[c]["ms"] / steps, 3) for c in pn if pn[c]["count"]}}
    ref_n = norms["ortho"]["norm"]
    for meth in norms:
        norms[meth]["rel_diff_vs_ortho"] = abs(norms[meth]["norm"] - ref_n) / ref_n
    return norms


def bench_sum3(h, ttr, torch, steps, warmup, I_n):
    """X = A + B + 1e-6 C (N=16, ranks 20 + 20 + 10 -> 50, 73.6 GB of cores at
    I = 262144), rounded at tol 1e-8 in FP64 and in mixed precision: the
    workload where the FP32 Gram passes must be refined to keep the 1e-6 part.
    Ranks and sampled entries of the mixed result are compared with FP64."""
    import synth
    torch.cuda.empty_cache()
    log("sum3: generating A, B, C (N=16, ranks 20, 20, 10)")
    d = synth.sum_r50(I_override=I_n)
    A, B, C = (ttr.TT.from_numpy(d[k]) for k in ("A", "B", "C"))
    tol = d["tol"]
    del d
    AB = h.add(1.0, A, 1.0, B)
    del A, B
    X = h.add(1.0, AB, 1.0, C)
    del AB, C
    torch.cuda.empty_cache()
    nbytes = sum(8 * X.R[n] * X.I[n] * X.R[n + 1] for n in range(X.N))
    Y = ttr.TT.empty(X.I, [X.R[n] * X.I[n] * X.R[n + 1] for n in range(X.N)])
    stream = torch.cuda.current_stream()
    res = {"workload": f"X = A + B + 1e-6 C, N=16, I={I_n}, A,B random TTs of rank 20 and C of rank 10 "
                       f"(scaled N(0,1) cores, C's first core times 1e-6), formal ranks 50, ttr_round tol {tol:g} RLR",
           "core_bytes_X": nbytes}
    ref = None
    for prec in ("fp64", "mixed"):
        for _ in range(warmup):
            Y = h.round(X, tol, "RLR", prec, out=Y)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for k in range(steps):
            ev[k][0].record(stream)
            Y = h.round(X, tol, "RLR", prec, out=Y)
            ev[k][1].record(stream)
        torch.cuda.synchronize()
        ms = sum(a.elapsed_time(b) for a, b in ev) / steps
        idx = np.random.default_rng(9).integers(0, I_n, size=(256, X.N))
        ent = sample_entries(Y.cores, list(Y.R), X.I, idx)
        r = {"ms_per_round": round(ms, 3), "round_core_GBps": round(nbytes / (ms * 1e-3) / 1e9, 2),
             "ranks": list(Y.R), "error_bound": error_bound_figures(h, torch, Y, tol)}
        if ref is None:
            ref = (list(Y.R), ent)
            r["ranks_ok"] = Y.R[1:-1] == [50] * (X.N - 1)
        else:
            r["ranks_equal_fp64"] = list(Y.R) == ref[0]
            r["max_entry_diff_vs_fp64"] = float(np.max(np.abs(ent - ref[1])) / np.sqrt(np.mean(ref[1] * ref[1])))
        res[prec] = r
        log(f"sum3 {prec}: {ms:.1f} ms per round")
    res["mixed_speedup"] = round(res["fp64"]["ms_per_round"] / res["mixed"]["ms_per_round"], 3)
    del X, Y
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--I", type=int, default=262144)
    ap.add_argument("--prec", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--direction", default="RLR", choices=["RLR", "LRL"])
    ap.add_argument("--cpu-sample-I", type=int, default=16384)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision rounds")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched rounding of 512 tensors")
    ap.add_argument("--no-large", action="store_true", help="skip the Hadamard -> rank-256 rounding")
    ap.add_argument("--no-norms", action="store_true", help="skip the timing of the three norm methods and of the explicit orthonormalization")
    ap.add_argument("--no-mirror", action="store_true",
                    help="skip the other rounding variants (mirror order, explicit orthonormal factors)")
    ap.add_argument("--no-sum3", action="store_true", help="skip the A + B + 1e-6 C rounding (ranks 50)")
    ap.add_argument("--leg", default="all", choices=["all", "batched", "large", "norms", "sum3"],
                    help="batched / large / norms / sum3: run only that leg (for profiling) and print its JSON object")
    ap.add_argument("--no-per-tensor", action="store_true",
                    help="batched leg: skip the one-ttr_round-per-tensor comparison")
    ap.add_argument("--copy-calibration", type=float, default=0.0,
                    help="only run a plain device-to-device copy of this many GiB (counter calibration)")
    args = ap.parse_args()

    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(sharding over several GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2011_06532_amd import ttr

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    h = ttr.Handle(0)

    if args.leg != "all":
        if args.leg == "batched":
            res = bench_batched(h, ttr, torch, args.steps, per_tensor=not args.no_per_tensor)
        elif args.leg == "sum3":
            res = bench_sum3(h, ttr, torch, args.steps, args.warmup, args.I)
        elif args.leg == "norms":
            d = synth.sum_r40(I_override=args.I)
            A, B = ttr.TT.from_numpy(d["A"]), ttr.TT.from_numpy(d["B"])
            del d
            X = h.add(1.0, A, 1.0, B)
            del A, B
            res = bench_norms(h, torch, X, sum(8 * X.R[n] * X.I[n] * X.R[n + 1] for n in range(len(X.I))),
                              args.steps)
        else:
            res = bench_large(h, ttr, torch, args.steps)
        h.close()
        print(json.dumps({"leg": args.leg, args.leg: res}), flush=True)
        return

    N, r = 16, 20
    log(f"generating A, B: N={N}, I={args.I}, ranks {r} (host, seeded)")
    t = time.perf_counter()
    d = synth.sum_r40(I_override=args.I)
    log(f"  generated in {time.perf_counter() - t:.1f} s; uploading")
    A = ttr.TT.from_numpy(d["A"])
    B = ttr.TT.from_numpy(d["B"])
    del d
    I = A.I
    RX = [1] + [A.R[n] + B.R[n] for n in range(1, N)] + [1]
    caps = [RX[n] * I[n] * RX[n + 1] for n in range(N)]
    Xbuf = ttr.TT.empty(I, caps)
    Ybuf = ttr.TT.empty(I, caps)
    size_x = sum(8 * c for c in caps)
    tol = synth.TOL[1]
    torch.cuda.synchronize()

    def step():
        X = h.add(1.0, A, 1.0, B, out=Xbuf)
        return X, h.round(X, tol, args.direction, args.prec, out=Ybuf)

    for w in range(args.warmup):
        log(f"warmup step {w + 1}/{args.warmup}")
        step()
    torch.cuda.synchronize()

    h.set_profiling(True)
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        e0, e1, e2 = ev[k]
        e0.record(stream)
        X = h.add(1.0, A, 1.0, B, out=Xbuf)
        e1.record(stream)
        Y = h.round(X, tol, args.direction, args.prec, out=Ybuf)
        e2.record(stream)
        log(f"step {k + 1}/{args.steps}")
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    prof = h.profile()
    h.set_profiling(False)
    st = h.round_stats()
    ms_step = sum(e0.elapsed_time(e2) for e0, _, e2 in ev) / args.steps
    ms_round = sum(e1.elapsed_time(e2) for _, e1, e2 in ev) / args.steps
    ms_add = sum(e0.elapsed_time(e1) for e0, e1, _ in ev) / args.steps
    ranks_ok = Y.R[1:-1] == [2 * r] * (N - 1)
    bound = error_bound_figures(h, torch, Y, tol) if args.direction == "RLR" else None
    Yf = [c.clone() for c in Y.cores]
    ranks_fp64 = list(Y.R)

    # the same rounding in mixed precision (FP32 first Gram passes), timed the
    # same way, and its result compared with the FP64 one through TT inner
    # products on the device
    mixed = None
    if args.prec == "fp64" and not args.no_mixed:
        log("mixed precision rounds")
        for w in range(args.warmup):
            Ym = h.round(Xbuf, tol, args.direction, "mixed", out=Ybuf)
        torch.cuda.synchronize()
        evm = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        for k in range(args.steps):
            evm[k][0].record(stream)
            Ym = h.round(Xbuf, tol, args.direction, "mixed", out=Ybuf)
            evm[k][1].record(stream)
        torch.cuda.synchronize()
        ms_mixed = sum(a.elapsed_time(b) for a, b in evm) / args.steps
        # entrywise agreement with the FP64 result on sampled multi-indices
        # (a norm of the difference would cancel at this size)
        idx = np.random.default_rng(7).integers(0, args.I, size=(256, N))
        ef = sample_entries(Yf, ranks_fp64, I, idx)
        em = sample_entries(Ym.cores, list(Ym.R), I, idx)
        rel = float(np.max(np.abs(em - ef)) / np.sqrt(np.mean(ef * ef)))
        mixed = {"ms_per_round": round(ms_mixed, 3),
                 "error_bound": error_bound_figures(h, torch, Ym, tol) if args.direction == "RLR" else None,
                 "round_core_GBps": round(size_x / (ms_mixed * 1e-3) / 1e9, 2),
                 "speedup_vs_fp64": round(ms_round / ms_mixed, 3),
                 "ranks_equal": list(Ym.R) == ranks_fp64,
                 "max_entry_diff_vs_fp64": rel,
                 "entries_sampled": int(idx.shape[0])}
        del Ym

    # the three norm methods of §3.2.4 on the same X
    norms = None if args.no_norms else bench_norms(h, torch, Xbuf, size_x, args.steps)

    # the other three rounding variants of §4.3.2 on the same X, FP64, timed
    # the same way: the mirror sweep order (LRL) and the explicit orthonormal
    # factors (cores written first, §3.4 Alg. 5) in both orders, with ranks
    # and sampled entries against this run's rounding
    mirror = None
    if args.prec == "fp64" and not args.no_mirror:
        mirror = {}
        other = "LRL" if args.direction == "RLR" else "RLR"
        for variant in (other, args.direction + "_EXPLICIT", other + "_EXPLICIT"):
            log(f"{variant} rounds")
            for w in range(args.warmup):
                Yo = h.round(Xbuf, tol, variant, "fp64", out=Ybuf)
            torch.cuda.synchronize()
            evo = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(args.steps)]
            for k in range(args.steps):
                evo[k][0].record(stream)
                Yo = h.round(Xbuf, tol, variant, "fp64", out=Ybuf)
                evo[k][1].record(stream)
            torch.cuda.synchronize()
            ms_o = sum(a.elapsed_time(b) for a, b in evo) / args.steps
            idx = np.random.default_rng(8).integers(0, args.I, size=(256, N))
            ef = sample_entries(Yf, ranks_fp64, I, idx)
            eo = sample_entries(Yo.cores, list(Yo.R), I, idx)
            mirror[variant] = {"ms_per_round": round(ms_o, 3),
                               "round_core_GBps": round(size_x / (ms_o * 1e-3) / 1e9, 2),
                               "ranks_equal": list(Yo.R) == ranks_fp64,
                               "max_entry_diff_vs_" + args.direction:
                                   float(np.max(np.abs(eo - ef)) / np.sqrt(np.mean(ef * ef)))}
            del Yo

    # explicit orthonormalization (orthonormal cores written, the §3.4 Alg. 5
    # form) of a copy of X, both sides; the implicit form is the first sweep
    # of every round (and the orthonormalization norm above)
    orth = None
    if not args.no_norms:
        log("explicit orthonormalization")
        orth = {}
        for side in ("right", "left"):
            ts, T = [], None
            for k in range(args.warmup + args.steps):
                for n in range(N):
                    m = RX[n] * I[n] * RX[n + 1]
                    Ybuf.cores[n][:m].copy_(Xbuf.cores[n][:m])
                T = ttr.TT(Ybuf.cores, I, RX)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                h.orthogonalize(T, side)
                e1.record(stream)
                torch.cuda.synchronize()
                if k >= args.warmup:
                    ts.append(e0.elapsed_time(e1))
            ms_t = sum(ts) / len(ts)
            # checks of the written cores: the core that carries the norm has
            # ||.||_F = the orthonormalization norm, and one interior core is
            # orthonormal (H H^T = I on the right side, V^T V = I on the left)
            nref = norms["ortho"]["norm"] if norms else h.norm(Xbuf, "ortho")
            c0 = 0 if side == "right" else N - 1
            m0 = T.R[c0] * I[c0] * T.R[c0 + 1]
            nc = float(torch.linalg.vector_norm(T.cores[c0][:m0]).item())
            mid = N // 2
            a, b = T.R[mid], T.R[mid + 1]
            core = T.cores[mid][:a * I[mid] * b]
            if side == "right":
                Hm = core.view(b * I[mid], a).t()          # H(X_n): a x (I b), column-major buffer
                gram = Hm @ Hm.t()
            else:
                Vm = core.view(b, a * I[mid]).t()          # V(X_n): (a I) x b
                gram = Vm.t() @ Vm
            orth_err = float(torch.linalg.matrix_norm(gram - torch.eye(gram.shape[0], dtype=gram.dtype,
                                                                          device=gram.device)).item())
            orth[side] = {"ms": round(ms_t, 3), "core_GBps": round(size_x / (ms_t * 1e-3) / 1e9, 2),
                          "ranks_kept": T.R == RX, "norm_core_rel_diff": abs(nc - nref) / nref,
                          "interior_core": mid, "interior_orthonormality": orth_err}
            del T  # it holds Ybuf's cores, which the later legs free

    # HBM fractions of the round against 8 TB/s: algorithmic bytes (X read
    # twice, the result written once) and, when the counter summary matches
    # the kernel sources, the measured bytes of the streaming kernels summed
    # over their launches
    size_y = sum(8 * ranks_fp64[n] * I[n] * ranks_fp64[n + 1] for n in range(N))
    hbm_frac = {"algorithmic": round((2 * size_x + size_y) / (ms_round * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
                "achieved": None}
    streamed = ("k_gram_right_factor", "k_gram_left_factor", "k_apply_mfma")
    per_launch = {c: pmc_traffic(c, 0.0) for c in streamed}
    if all(per_launch[c] is not None for c in streamed):
        tb = sum(per_launch[c] * prof[c]["count"] / args.steps for c in streamed)
        hbm_frac["achieved"] = round(tb / (ms_round * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)
        hbm_frac["achieved_bytes_per_round"] = round(tb)

    # dominant kernel by time
    cls = max((c for c in prof if c != "small"), key=lambda c: prof[c]["ms"])
    p = prof[cls]
    n_launch = max(p["count"], 1)
    ai = p["flops"] / p["bytes"] if p["bytes"] else 0.0
    if ai > RIDGE:
        achieved = p["flops"] / (p["ms"] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP64_PEAK_TFLOPS, 4)}
    else:
        achieved = p["bytes"] / (p["ms"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4)}
    roof["traffic"] = pmc_traffic(cls, p["bytes"] / n_launch)
    roof["kernel"] = cls
    roof["launches"] = p["count"]
    roof["avg_launch_ms"] = round(p["ms"] / n_launch, 4)
    roof["algorithmic_bytes_per_launch"] = round(p["bytes"] / n_launch)
    roof["algorithmic_flops_per_launch"] = round(p["flops"] / n_launch)
    roof["share_of_step"] = round(p["ms"] / args.steps / ms_step, 3)

    out = {
        "metric": "TT-round core-GB/s and ms/round, FP64 vs mixed at rel.err <=1e-8, 1 GPU",
        "value": round(size_x / (ms_round * 1e-3) / 1e9, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"X = A + B, N={N}, I={args.I}, A,B random TTs of rank {r} with N(0,1) cores "
                               f"scaled by 1/sqrt(R_(n-1) I_n), formal ranks {2 * r}, ttr_round tol {tol} "
                               f"{args.direction} {args.prec}",
                   "core_bytes_X": size_x},
        "ms_per_round": round(ms_round, 3),
        "ms_per_add": round(ms_add, 3),
        "step_core_GBps": round(size_x / (ms_step * 1e-3) / 1e9, 2),
        "error_bound": bound,
        "round_core_GBps": round(size_x / (ms_round * 1e-3) / 1e9, 2),
        "hbm_fraction": hbm_frac,
        "wall_ms_per_step": round(wall * 1e3, 3),
        "ranks_ok": ranks_ok,
        "gram_passes": st["gram_passes"],
        "apply_passes": st["apply_passes"],
        "kernel_ms_per_step": {c: round(prof[c]["ms"] / args.steps, 3) for c in prof if prof[c]["count"]},
        "roofline": roof,
    }
    if mixed:
        out["mixed"] = mixed
    if norms:
        out["norms"] = norms
    if mirror:
        out["rounding_variants"] = mirror
    if orth:
        out["orthogonalize_explicit"] = orth
    del A, B, Xbuf, Ybuf, X, Y, Yf
    torch.cuda.empty_cache()
    if not args.no_sum3:
        out["sum3"] = bench_sum3(h, ttr, torch, args.steps, args.warmup, args.I)
    if not args.no_batched:
        out["batched"] = bench_batched(h, ttr, torch, args.steps, per_tensor=not args.no_per_tensor)
    if not args.no_large:
        # a fresh handle: the workspaces the earlier legs grew (materialized
        # cores, batched plans) go back to the device, so this leg has the
        # memory a run of its own has (the rank-256 rounding keeps the first
        # sweep's products when they fit)
        h.close()
        h = ttr.Handle(0)
        out["large"] = bench_large(h, ttr, torch, args.steps)
    if not args.no_cpu_baseline:
        log(f"cpu_baseline: oracle on I={args.cpu_sample_I}")
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample_I)
    h.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
