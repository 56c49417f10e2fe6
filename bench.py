"""Throughput bench for decentralized detection / precoding on one MI355X.

A step is one pass of the whole detection path -- load H and y, per-cluster Gram
and regularised inverse, T decentralized ADMM iterations with their consensus
sums, slicing -- over one launch of 32 frames x 1200 subcarriers (38,400
independent subcarrier-vectors, each with its own channel; the paper's GPU
batches 1200 x 7 vectors), followed by the FP64 re-slice pass over the
subcarriers it flagged.  Single-frame (1200-subcarrier) launch latency is
reported beside it, and the serving run reports latency under load.  The default workload is
decentralized ADMM uplink detection (Algorithm 1) at B=256 antennas, U=32
users, C=8 clusters (S=32), 64-QAM, 25 dB, rho=1, T=5, N_sym=1.  Frames are
synthetic i.i.d. Rayleigh (generated on the device from a fixed seed) and stay
resident in HBM; consecutive steps rotate over more distinct frames than the
Infinity Cache holds, so every H byte is read from HBM.

Prints one JSON line (rank 0).  ``--gpus`` above 1 is refused: the benchmark
measures one GPU's share of the work.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, published
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector, published
FP32_MFMA_PEAK_TFLOPS = 157.3
FP16_MFMA_PEAK_TFLOPS = 2500.0

DEFAULT_FRAMES_PER_STEP = 32     # frames of one workload per timed launch

WORKLOADS = {
    # name: (algo, B, U, C, qam, snr_db, T, n_sc)
    "admm_ul_B256_U32_C8": ("admm", 256, 32, 8, 64, 25.0, 5, 1200),
    "admm_ul_B256_U32_C4": ("admm", 256, 32, 4, 64, 25.0, 5, 1200),
    "admm_ul_B128_U16_C8": ("admm", 128, 16, 8, 16, 10.0, 5, 1200),
    "dcg_ul_B128_U16_C8": ("cg", 128, 16, 8, 16, 10.0, 5, 1200),
    "admm_dl_B256_U32_C16": ("dl", 256, 32, 16, 64, 0.0, 5, 1200),
    "admm_ul_B512_U64_C8": ("admm", 512, 64, 8, 64, 25.0, 5, 1200),
}


def algorithmic_bytes(algo, B, U, C, form="oneshot"):
    """HBM bytes one subcarrier-vector must move (complex64 in/out, uint8 hard).
    The resident forms also read the factors B_c^{-1} (complex64, the upper
    triangle of each Hermitian block); the FP16 channel holds H in 4 bytes per
    entry plus one float scale per cluster."""
    if algo == "dl":
        return 8 * B * U + 8 * U + 8 * B
    if form == "resident":
        return 8 * B * U + 8 * C * (U * (U + 1) // 2) + 8 * B + 8 * U + U
    if form == "resident_h16":
        return 4 * B * U + 4 * C + 8 * C * (U * (U + 1) // 2) + 8 * B + 8 * U + U
    return 8 * B * U + 8 * B + 8 * U + U


def algorithmic_flops(algo, B, U, C, T, form="oneshot"):
    """Minimal real flops per vector (complex MAC = 8 flops; Hermitian Gram at
    half cost; factorisation U^3/6 complex MACs; one U^2 solve per estimate).
    The resident forms form no Gram and no factorisation."""
    S = B // C
    if algo == "admm" and form != "oneshot":
        return 8.0 * (B * U + C * U * U + (T - 1) * C * U * U)
    if algo == "admm":
        cm = C * S * U * (U + 1) / 2 + C * U ** 3 / 6 + B * U + C * U * U + (T - 1) * C * U * U
    elif algo == "cg":
        cm = B * U * (1 + 2 * T)
    else:
        cm = C * U * S * (S + 1) / 2 + C * S ** 3 / 6 + C * (S * U + S * S) + (T - 1) * C * (2 * S * U + S * S)
    return 8.0 * cm


def make_frames(n_frames, algo, B, U, qam, snr_db, n_sc, seed):
    """Seeded synthetic frames generated on the device: H ~ CN(0,1) i.i.d.,
    unit-energy QAM symbols, AWGN with N0 = U / SNR (same recipe as
    paper_1702_04458_amd.inputs)."""
    import torch

    from paper_1702_04458_amd import inputs

    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    L = inputs.qam_side(qam)
    kappa = inputs.qam_kappa(qam)
    N0 = U / (10.0 ** (snr_db / 10.0))
    frames = []
    for _ in range(n_frames):
        H = torch.complex(torch.randn((n_sc, B, U), generator=g, device="cuda"),
                          torch.randn((n_sc, B, U), generator=g, device="cuda")) / math.sqrt(2.0)
        iI = torch.randint(0, L, (n_sc, 1, U), generator=g, device="cuda")
        iQ = torch.randint(0, L, (n_sc, 1, U), generator=g, device="cuda")
        s = torch.complex((2 * iI - (L - 1)).float(), (2 * iQ - (L - 1)).float()) / kappa
        if algo == "dl":
            frames.append((H.contiguous(), s.contiguous()))
            continue
        n = torch.complex(torch.randn((n_sc, 1, B), generator=g, device="cuda"),
                          torch.randn((n_sc, 1, B), generator=g, device="cuda")) * math.sqrt(N0 / 2.0)
        y = torch.matmul(H, s.transpose(1, 2).contiguous()).transpose(1, 2) + n
        frames.append((H.contiguous(), y.contiguous()))
    return frames, N0


_WS = {}


def _ws(api, n_sc, U, C):
    """One FP64 re-slice workspace per shape, allocated once outside the timed steps."""
    key = (n_sc, U, C)
    if key not in _WS:
        _WS[key] = api.workspace(n_sc, U, C)
    return _WS[key]


def received_over(H, n_frames, qam, snr_db, seed):
    """Received frames y = H s + n over one static channel H [n_sc, B, U]
    (fresh symbols and noise per frame, same recipe as make_frames): the
    workload of the resident (static-channel) forms."""
    import torch

    from paper_1702_04458_amd import inputs

    n_sc, B, U = H.shape
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    L = inputs.qam_side(qam)
    kappa = inputs.qam_kappa(qam)
    N0 = U / (10.0 ** (snr_db / 10.0))
    ys = []
    for _ in range(n_frames):
        iI = torch.randint(0, L, (n_sc, 1, U), generator=g, device="cuda")
        iQ = torch.randint(0, L, (n_sc, 1, U), generator=g, device="cuda")
        s = torch.complex((2 * iI - (L - 1)).float(), (2 * iQ - (L - 1)).float()) / kappa
        n = torch.complex(torch.randn((n_sc, 1, B), generator=g, device="cuda"),
                          torch.randn((n_sc, 1, B), generator=g, device="cuda")) * math.sqrt(N0 / 2.0)
        ys.append((torch.matmul(H, s.transpose(1, 2).contiguous()).transpose(1, 2) + n).contiguous())
    return ys


def run_step(api, frame, algo, C, T, N0, qam, out, prec="fp32", factor=None, resident=None):
    """One detection call over one step's subcarriers (the FP32 kernel, then
    the FP64 re-slice pass over its flags).  ``resident`` = (form, channel
    state, factors, B, U) runs the resident form against the frame's y only."""
    n_sc, U = out[0].shape[0], out[0].shape[2]
    if resident is not None:
        form, chan, fac, B, U = resident
        if form == "resident":
            api.detect_factored(chan, fac, frame[1], N0, C, 1.0, T, qam=qam, out=out, workspace=_ws(api, n_sc, U, C))
        else:
            api.detect_factored_h16(chan, fac, frame[1], N0, B, U, C, 1.0, T, qam=qam, out=out)
        return
    if algo == "dl":
        api.precode(frame[0], frame[1], C, 1.0, T, out=out)
    else:
        api.detect(frame[0], frame[1], N0, C, 1.0, T, algo=algo, qam=qam, out=out, prec=prec, factor=factor,
                   workspace=_ws(api, n_sc, U, C))


def _blas_threads():
    """BLAS / OpenMP threads numpy actually uses in this process (threadpoolctl)."""
    try:
        from threadpoolctl import threadpool_info
        return max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    except Exception:
        return None


def _oracle_worker(args):
    from oracle import dbp_oracle as O
    from paper_1702_04458_amd import inputs

    algo, B, U, C, qam, snr, T, seed, budget_s = args
    t0 = time.perf_counter()
    done = 0
    k = 0
    busy = 0.0          # oracle time only: input generation is excluded
    while time.perf_counter() - t0 < budget_s:
        if algo == "dl":
            fr = inputs.downlink_frame(seed + k, 4, B, U, qam)
            t1 = time.perf_counter()
            O.admm_dl_frame(fr.H, fr.s, C, 1.0, T)
        else:
            fr = inputs.uplink_frame(seed + k, 4, B, U, qam, snr)
            t1 = time.perf_counter()
            if algo == "admm":
                O.admm_ul_frame(fr.H, fr.y, C, 1.0, T, fr.N0)
            else:
                O.dcg_ul_frame(fr.H, fr.y, C, T, fr.N0)
        busy += time.perf_counter() - t1
        done += 4
        k += 1
    return done, busy, _blas_threads()


def host_info():
    """Logical CPUs of the host, CPUs this process may run on, CPU model."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"nproc": os.cpu_count() or 1, "usable_cpus": usable, "cpu_model": model}


# The GPU host gives one GPU's job a share of 16 CPU cores, whatever the
# machine's core count: the process pools below use at most that many.
CPU_SHARE = 16


def _single_thread_pool(workers):
    """A spawn pool whose workers start with one BLAS / OpenMP thread each (the
    variables are set before the workers import numpy)."""
    import multiprocessing as mp

    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    try:
        pool = mp.get_context("spawn").Pool(workers)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return pool


def cpu_baseline(algo, B, U, C, qam, snr, T, budget_s=12.0):
    """FP64 oracle on the host cores, subcarrier-parallel over worker processes
    (one BLAS thread each, CPU_SHARE processes at most); input generation is
    excluded from the measured time."""
    host = host_info()
    workers = max(1, min(host["usable_cpus"], CPU_SHARE))
    t0 = time.perf_counter()
    with _single_thread_pool(workers) as pool:
        res = pool.map(_oracle_worker, [(algo, B, U, C, qam, snr, T, 5000 + 97 * i, budget_s) for i in range(workers)])
    wall = time.perf_counter() - t0
    vecs = sum(r[0] for r in res)
    # every worker runs for the same wall budget; the aggregate rate sums the
    # workers' own rates (oracle time only, input generation excluded)
    value = sum(r[0] / r[1] for r in res)
    out = {"value": value, "unit": "vectors/s", "cores": workers, "kind": "oracle",
           "per_core_value": value / workers, "threads_per_process": max(r[2] or 1 for r in res),
           "host_nproc": host["nproc"], "host_usable_cpus": host["usable_cpus"], "cpu_model": host["cpu_model"],
           "sample": f"{vecs} subcarrier-vectors of the same shape (fresh seeded frames), "
                     f"{workers} worker processes (the {CPU_SHARE}-core CPU share of one GPU) x {budget_s:.0f} s, "
                     f"FP64 numpy oracle, input generation excluded; wall {wall:.1f} s"}
    if algo == "admm":
        out["vectorized"] = cpu_vectorized_admm(B, U, C, qam, snr, T, workers)
    return out


def _vectorized_worker(args):
    """Batched numpy form of Algorithm 1 (U x U branch, MMSE, rho = 1) over a
    whole frame in FP64: batched inverses of all B_c, then T iterations as
    batched matrix-vector products.  Measurement aid only (not the oracle);
    checked against the oracle on a few subcarriers before timing.  Returns
    (vectors, seconds, BLAS threads)."""
    import numpy as np

    from oracle import dbp_oracle as O
    from paper_1702_04458_amd import inputs

    B, U, C, qam, snr, T, n_sc, reps, seed = args
    S = B // C
    fr = inputs.uplink_frame(seed, n_sc, B, U, qam, snr)
    H = fr.H.astype(np.complex128).reshape(n_sc, C, S, U)
    y = fr.y[:, 0].astype(np.complex128).reshape(n_sc, C, S)
    den = fr.N0 + C            # N0 / (rho Es) + C with rho = Es = 1

    def run():
        Hh = np.conj(np.swapaxes(H, -1, -2))                             # [n_sc, C, U, S]
        Binv = np.linalg.inv(Hh @ H + np.eye(U))                         # rho = 1
        yreg = (Binv @ (Hh @ y[..., None]))[..., 0]                      # [n_sc, C, U]
        z, lam = yreg, np.zeros_like(yreg)
        s = z.sum(axis=1) / den
        for _ in range(2, T + 1):
            lam = lam + (z - s[:, None])
            z = yreg + (Binv @ (s[:, None] - lam)[..., None])[..., 0]
            s = (z + lam).sum(axis=1) / den
        return s

    s = run()
    ref = O.admm_ul_frame(fr.H[:4], fr.y[:4], C, 1.0, T, fr.N0)[:, 0]
    assert np.abs(s[:4] - ref).max() <= 1e-9 * np.abs(ref).max()
    t0 = time.perf_counter()
    for _ in range(reps):
        run()
    return n_sc * reps, time.perf_counter() - t0, _blas_threads()


def cpu_vectorized_admm(B, U, C, qam, snr, T, workers, n_sc=1200, reps=3):
    """The batched form over `workers` processes with one BLAS thread each (its
    small batched matrices gain nothing from threads inside one process), each
    on its own frame; the rate sums the workers' own rates."""
    with _single_thread_pool(workers) as pool:
        res = pool.map(_vectorized_worker, [(B, U, C, qam, snr, T, n_sc, reps, 777 + i) for i in range(workers)])
    value = sum(r[0] / r[1] for r in res)
    return {"value": round(value, 1), "unit": "vectors/s", "processes": workers,
            "threads_per_process": max(r[2] or 1 for r in res),
            "per_process_value": round(value / workers, 1),
            "sample": f"{workers} processes x {n_sc} subcarriers x {reps} repetitions, FP64, batched numpy "
                      f"(not the oracle)"}


def _pctl(v, q):
    v = sorted(v)
    return v[min(len(v) - 1, max(0, int(math.ceil(q * len(v))) - 1))]


def serve_bench(loads=(0.25, 0.5, 0.7, 0.85, 0.95), frames_per_load=10000, pool=40, n_slots=8,
                budget_gb=32.0, seed=99, max_batch=8, log=sys.stderr):
    """Continuous-batching serving run: Poisson arrivals of uplink frames whose
    (B, U, C) is uniform over the valid triples with U <= S = B/C, n_sc uniform
    over {72, 300, 600, 1200}, 16/64-QAM, SNR 0..20 dB, ADMM (rho=1, T=5).
    Frames are resident in HBM (device I/O mode).  Returns saturation
    throughput and per-load p50/p99 latency (submit to completion)."""
    import random
    import threading

    import torch

    from paper_1702_04458_amd import api, inputs

    rng = random.Random(seed)
    shapes = inputs.serving_shapes()
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    frames = []
    for i in range(pool):
        B, U, C = rng.choice(shapes)
        n_sc = rng.choice((72, 300, 600, 1200))
        qam = rng.choice((16, 64))
        snr = rng.choice((0, 5, 10, 15, 20))
        N0 = U / (10.0 ** (snr / 10.0))
        H = torch.complex(torch.randn((n_sc, B, U), generator=g, device="cuda"),
                          torch.randn((n_sc, B, U), generator=g, device="cuda")) / math.sqrt(2.0)
        L = inputs.qam_side(qam)
        kap = inputs.qam_kappa(qam)
        iI = torch.randint(0, L, (n_sc, U, 1), generator=g, device="cuda")
        iQ = torch.randint(0, L, (n_sc, U, 1), generator=g, device="cuda")
        sv = torch.complex((2 * iI - (L - 1)).float(), (2 * iQ - (L - 1)).float()) / kap
        nse = torch.complex(torch.randn((n_sc, B, 1), generator=g, device="cuda"),
                            torch.randn((n_sc, B, 1), generator=g, device="cuda")) * math.sqrt(N0 / 2.0)
        y = (torch.matmul(H, sv) + nse).transpose(1, 2).contiguous()
        frames.append(dict(H=H.contiguous(), y=y, B=B, U=U, C=C, n_sc=n_sc, qam=qam, N0=N0))
    torch.cuda.synchronize()
    srv = api.Server(hbm_budget_bytes=int(budget_gb * 2 ** 30), n_slots=n_slots)
    srv.set_batching(max_batch)

    def outs(f):
        return (torch.empty((f["n_sc"], 1, f["U"]), dtype=torch.complex64, device="cuda"),
                torch.empty((f["n_sc"], 1, f["U"]), dtype=torch.uint8, device="cuda"))

    out_pool = [outs(f) for f in frames]

    def submit(i):
        f = frames[i % pool]
        o = out_pool[i % pool]
        return srv.submit(f["H"], f["y"], o[0], o[1], f["C"], 5, 1.0, f["N0"], qam=f["qam"])

    # warm up every shape once
    for t in [submit(i) for i in range(pool)]:
        srv.wait(t)
    # saturation: closed loop, everything queued at once
    n_sat = 4 * pool
    t0 = time.perf_counter()
    tickets = [submit(i) for i in range(n_sat)]
    for t in tickets:
        srv.wait(t)
    sat_fps = n_sat / (time.perf_counter() - t0)
    vec_per_frame = sum(f["n_sc"] for f in frames) / pool
    print(f"[serve] saturation {sat_fps:.0f} frames/s ({sat_fps * vec_per_frame / 1e6:.2f} M vectors/s)",
          file=log, flush=True)
    results = []
    for load in loads:
        rate = load * sat_fps
        lat = []
        pend = []
        lock = threading.Lock()
        done_flag = [False]

        def waiter():
            while True:
                with lock:
                    item = pend.pop(0) if pend else None
                if item is None:
                    if done_flag[0]:
                        with lock:
                            if not pend:
                                return
                    time.sleep(0.0002)
                    continue
                lat.append(srv.wait(item)[0])

        th = threading.Thread(target=waiter)
        th.start()
        t_next = time.perf_counter()
        t_start = t_next
        for i in range(frames_per_load):
            t_next += rng.expovariate(rate)
            while time.perf_counter() < t_next:
                pass
            tk = submit(rng.randrange(pool))
            with lock:
                pend.append(tk)
        done_flag[0] = True
        th.join()
        dur = time.perf_counter() - t_start
        lat.sort()
        p50 = lat[len(lat) // 2]
        p99 = lat[min(len(lat) - 1, int(math.ceil(0.99 * len(lat))) - 1)]
        results.append({"load": load, "offered_fps": round(rate, 1), "achieved_fps": round(len(lat) / dur, 1),
                        "p50_us": round(p50, 1), "p99_us": round(p99, 1), "frames": len(lat)})
        print(f"[serve] load {load:.2f}: p50 {p50:.0f} us, p99 {p99:.0f} us", file=log, flush=True)
    st = srv.stats()
    srv.close()
    return {"saturation_fps": round(sat_fps, 1), "max_batch": max_batch,
            "saturation_vectors_per_s": round(sat_fps * vec_per_frame, 1),
            "mean_subcarriers_per_frame": round(vec_per_frame, 1), "slots": n_slots, "budget_gb": budget_gb,
            "peak_inflight": st["peak_inflight"], "loads": results}


def serve_h16_bench(api, F=7, loads=(0.5, 0.85), intervals_per_load=600, n_channels=8, B=256, U=32, C=8,
                    n_sc=1200, qam=64, snr=25.0, n_slots=8, budget_gb=32.0, seed=7, log=sys.stderr):
    """The mixed-precision served form under Poisson arrivals: uplink frames
    over static channels, F frames per channel (a coherence interval of F
    OFDM symbols).  The first frame of every interval loads its channel into
    the server (dbp_channel_load with DBP_CHANNEL_H16: H packed as complex
    FP16 and B_c^{-1} formed once), the F frames run the FP32 iterations
    against it (dbp_server_submit_factored), and the channel is freed once
    its frames are done.  A frame's latency runs from its Poisson arrival to
    its completion, so the channel load and any queueing count.  Saturation
    is measured closed-loop first."""
    import random
    import threading

    import torch

    rng = random.Random(seed)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    Hs = [(torch.complex(torch.randn((n_sc, B, U), generator=g, device="cuda"),
                         torch.randn((n_sc, B, U), generator=g, device="cuda")) / math.sqrt(2.0)).contiguous()
          for _ in range(n_channels)]
    ys = [received_over(H, F, qam, snr, seed + 1 + i) for i, H in enumerate(Hs)]
    N0 = U / (10.0 ** (snr / 10.0))
    outs = [[(torch.empty((n_sc, 1, U), dtype=torch.complex64, device="cuda"),
              torch.empty((n_sc, 1, U), dtype=torch.uint8, device="cuda")) for _ in range(F)]
            for _ in range(n_channels)]
    torch.cuda.synchronize()
    srv = api.Server(hbm_budget_bytes=int(budget_gb * 2 ** 30), n_slots=n_slots)

    def run(n_intervals, rate):
        """rate None: closed loop.  Returns (frames, seconds, latencies_us)."""
        lat = []
        pend = []             # (arrival, submit, ticket, interval)
        lock = threading.Lock()
        state = {"done": False}
        left = {}             # interval -> frames not yet completed
        chans = {}

        def waiter():
            while True:
                with lock:
                    item = pend.pop(0) if pend else None
                if item is None:
                    if state["done"]:
                        with lock:
                            if not pend:
                                return
                    time.sleep(0.0001)
                    continue
                arr, sub, tk, iv = item
                l_us, _ = srv.wait(tk)
                lat.append((sub - arr) * 1e6 + l_us)
                with lock:
                    left[iv] -= 1
                    free = left[iv] == 0
                if free:
                    srv.free_channel(chans.pop(iv))

        th = threading.Thread(target=waiter)
        th.start()
        t0 = time.perf_counter()
        t_next = t0
        for iv in range(n_intervals):
            ci = iv % n_channels
            for f in range(F):
                if rate is not None:
                    t_next += rng.expovariate(rate)
                    while time.perf_counter() < t_next:
                        pass
                arr = t_next if rate is not None else time.perf_counter()
                if f == 0:
                    # keep at most n_channels - 1 intervals resident (their buffers are reused)
                    while True:
                        with lock:
                            busy = len(chans)
                        if busy < n_channels - 1:
                            break
                        time.sleep(0.00005)
                    ch = srv.load_channel(Hs[ci], C, 1.0, h16=True)
                    with lock:
                        chans[iv] = ch
                        left[iv] = F
                o = outs[ci][f]
                tk = srv.submit_factored(chans[iv], ys[ci][f], o[0], o[1], 5, N0, qam=qam)
                with lock:
                    pend.append((arr, time.perf_counter(), tk, iv))
        state["done"] = True
        th.join()
        return n_intervals * F, time.perf_counter() - t0, lat

    run(2 * n_channels, None)                                   # warm-up
    nf, dt, _ = run(max(40, intervals_per_load // 4), None)
    sat_fps = nf / dt
    print(f"[serve-h16] saturation {sat_fps:.0f} frames/s ({sat_fps * n_sc / 1e6:.2f} M vectors/s)", file=log,
          flush=True)
    res = []
    for load in loads:
        nf, dt, lat = run(intervals_per_load, load * sat_fps)
        res.append({"load": load, "offered_fps": round(load * sat_fps, 1), "achieved_fps": round(nf / dt, 1),
                    "vectors_per_s": round(nf * n_sc / dt, 1), "p50_us": round(_pctl(lat, 0.5), 1),
                    "p99_us": round(_pctl(lat, 0.99), 1), "frames": nf})
        print(f"[serve-h16] load {load:.2f}: p50 {res[-1]['p50_us']:.0f} us, p99 {res[-1]['p99_us']:.0f} us",
              file=log, flush=True)
    srv.close()
    return {"shape": f"B={B} U={U} C={C} n_sc={n_sc} {qam}-QAM {snr:g} dB T=5", "frames_per_channel": F,
            "saturation_fps": round(sat_fps, 1), "saturation_vectors_per_s": round(sat_fps * n_sc, 1),
            "loads": res}


def nsym_bench(api, B, U, C, qam, snr, T, n_sym=7, n_vectors=38400, steps=30, log=sys.stderr):
    """The static-channel GPU workload of the paper's measurements: N_sym
    received vectors per subcarrier share one channel, so one launch forms
    every B_c^{-1} once and runs Algorithm 1 for all N_sym symbols."""
    import torch

    n_sc = n_vectors // n_sym
    frames = []
    for i in range(3):
        H = make_frames(1, "admm", B, U, qam, snr, n_sc, seed=555 + i)[0][0][0]
        ys = received_over(H, n_sym, qam, snr, seed=777 + i)
        frames.append((H, torch.cat(ys, dim=1).contiguous()))
    out = (torch.empty((n_sc, n_sym, U), dtype=torch.complex64, device="cuda"),
           torch.empty((n_sc, n_sym, U), dtype=torch.uint8, device="cuda"))
    N0 = U / (10.0 ** (snr / 10.0))
    ms, per = time_steps(api, frames, "admm", C, T, N0, qam, out, "fp32", None, steps, 5)
    vec = n_sc * n_sym
    bytes_vec = (8 * B * U + n_sym * (8 * B + 8 * U + U)) / n_sym
    avg_ms = sum(per) / len(per)
    print(f"[bench] N_sym={n_sym}: {ms * 1e3:.1f} us/step, {vec / (ms * 1e-3) / 1e6:.1f} M vectors/s", file=log,
          flush=True)
    return {"n_sym": n_sym, "n_sc": n_sc, "vectors": vec, "us_per_step": round(ms * 1e3, 2),
            "vectors_per_s": round(vec / (ms * 1e-3), 1), "bytes_per_vector": round(bytes_vec, 1),
            "hbm_frac": round(bytes_vec * vec / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def dl_budget_bench(api, frames, C, T, out, steps, P=0.013, log=sys.stderr):
    """Configuration 3 with per-cluster budgets P_c (binding on about half of
    the clusters at this shape): the common gain after Algorithm 3, and the
    budgeted step (P1) in every x-update."""
    import torch

    res = {"P_c": P}
    Pt = torch.full((C,), P, dtype=torch.float32, device="cuda")
    for mode in ("common_gain", "per_cluster"):
        for i in range(3):
            api.precode(frames[i % len(frames)][0], frames[i % len(frames)][1], C, 1.0, T, P_cluster=Pt, power=mode,
                        out=out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for i in range(steps):
            api.precode(frames[i % len(frames)][0], frames[i % len(frames)][1], C, 1.0, T, P_cluster=Pt, power=mode,
                        out=out)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        n_sc = frames[0][0].shape[0]
        res[mode] = {"us_per_step": round(ms * 1e3, 2), "vectors_per_s": round(n_sc / (ms * 1e-3), 1)}
        print(f"[bench] downlink budget {mode}: {ms * 1e3:.1f} us/step", file=log, flush=True)
    return res


def source_digest() -> str:
    """sha256 over the HIP sources: identifies the kernel build a profile was taken on."""
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1702_04458_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h", ".cpp")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode())
                h.update(f.read())
    return h.hexdigest()


def profiled_traffic(workload: str):
    """HBM bytes per launch recorded in profiles/<workload>.md (FETCH_SIZE and
    WRITE_SIZE, calibrated against a device copy), if that profile was taken on
    the current kernel sources; otherwise None."""
    path = os.path.join(ROOT, "profiles", f"{workload}.md")
    if not os.path.exists(path):
        return None
    digest, traffic = None, None
    with open(path) as f:
        for line in f:
            if line.startswith("source-sha256:"):
                digest = line.split(":", 1)[1].strip()
            if line.startswith("hbm-bytes-per-launch:"):
                traffic = float(line.split(":", 1)[1].strip())
    if digest != source_digest():
        return None
    return traffic


def time_steps(api, frames, algo, C, T, N0, qam, out, prec, factor, steps, warmup, n_streams=1, resident=None):
    """Runs warmup + steps launches rotating over the resident frames; returns
    (ms per step from the events bracketing all steps, sorted per-launch ms).
    With n_streams > 1 consecutive frames go to different streams (each with
    its own output buffers), so one frame's tail overlaps the next frame's start,
    as in a pipelined frame-by-frame receiver."""
    import torch

    n_frames = len(frames)
    main = torch.cuda.current_stream()
    streams = [main] + [torch.cuda.Stream() for _ in range(n_streams - 1)]
    outs = [out] + [tuple(torch.empty_like(t) for t in out) for _ in range(n_streams - 1)]
    for i in range(warmup):
        run_step(api, frames[i % n_frames], algo, C, T, N0, qam, out, prec, factor, resident)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    start_all = torch.cuda.Event(enable_timing=True)
    end_all = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start_all.record(main)
    for st in streams[1:]:
        st.wait_event(start_all)
    for i in range(steps):
        j = i % n_streams
        with torch.cuda.stream(streams[j]):
            ev[i][0].record(streams[j])
            run_step(api, frames[i % n_frames], algo, C, T, N0, qam, outs[j], prec, factor, resident)
            ev[i][1].record(streams[j])
    for st in streams[1:]:
        main.wait_stream(st)
    end_all.record(main)
    torch.cuda.synchronize()
    per = sorted(e[0].elapsed_time(e[1]) for e in ev)
    return start_all.elapsed_time(end_all) / steps, per


def mixed_cfg4_bench(api, n_sc=9600, steps=10, warmup=2, log=sys.stderr):
    """Configuration 4 (B=512, C=8, S=64, U=64, 64-QAM, 25 dB, T=5): the FP32
    path against the mixed modes, one-shot, exact hard decisions, 9,600
    subcarriers per launch (two resident frames)."""
    import torch
    B, U, C, qam, snr, T = 512, 64, 8, 64, 25.0, 5
    frames, N0 = make_frames(2, "admm", B, U, qam, snr, n_sc, seed=4404)
    out = (torch.empty((n_sc, 1, U), dtype=torch.complex64, device="cuda"),
           torch.empty((n_sc, 1, U), dtype=torch.uint8, device="cuda"))
    res = {"shape": f"B={B} U={U} C={C} {qam}-QAM {snr:g} dB T={T}", "n_sc": n_sc}
    for prec, factor in (("fp32", None), ("fp16", "auto"), ("fp16", "f16x2"), ("bf16", "auto")):
        ms, _ = time_steps(api, frames, "admm", C, T, N0, qam, out, prec, factor, steps, warmup)
        key = "fp32" if prec == "fp32" else f"{prec}_factor_{factor}"
        res[key] = {"us_per_step": round(ms * 1e3, 1), "vectors_per_s": round(n_sc / (ms * 1e-3), 1)}
        print(f"[bench] configuration 4 {key}: {ms * 1e3:.1f} us/step", file=log, flush=True)
    base = res["fp32"]["vectors_per_s"]
    res["rule_mixed_vs_fp32"] = round(res["fp16_factor_auto"]["vectors_per_s"] / base, 3)
    res["best_mixed_vs_fp32"] = round(max(v["vectors_per_s"] for k, v in res.items()
                                          if isinstance(v, dict) and k != "fp32") / base, 3)
    del frames
    torch.cuda.empty_cache()
    return res


def static_channel_bench(api, frames, C, T, N0, qam, snr_db, out, steps):
    """Static channel over the coherence interval: B_c^{-1} is formed once per
    channel (dbp_factor_admm) and every received frame runs only Algorithm 1's
    iterations against it (dbp_detect_admm_factored).  Times the factorisation
    and the factored detection of one step's subcarriers; the received frames
    are generated over that one channel."""
    import torch

    H0 = frames[0][0]
    ys = received_over(H0, 4, qam, snr_db, seed=4321)
    frames = [(H0, y) for y in ys]
    n_sc = H0.shape[0]
    fac = api.factor(H0, C, 1.0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        api.factor(H0, C, 1.0, out=fac)
    e1.record()
    torch.cuda.synchronize()
    factor_ms = e0.elapsed_time(e1) / 5
    ws = _ws(api, n_sc, H0.shape[2], C)
    for i in range(3):
        api.detect_factored(H0, fac, frames[i % len(frames)][1], N0, C, 1.0, T, qam=qam, out=out, workspace=ws)
    torch.cuda.synchronize()
    e0.record()
    for i in range(steps):
        api.detect_factored(H0, fac, frames[i % len(frames)][1], N0, C, 1.0, T, qam=qam, out=out, workspace=ws)
    e1.record()
    torch.cuda.synchronize()
    det_ms = e0.elapsed_time(e1) / steps
    # mixed-precision resident form: H packed as complex FP16 (per-tile
    # power-of-two scale), FP32 factors, FP32 iterations
    B, U = H0.shape[1], H0.shape[2]
    packed = api.pack_channel_h16(H0, C)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(5):
        api.pack_channel_h16(H0, C, out=packed)
    e1.record()
    torch.cuda.synchronize()
    pack_ms = e0.elapsed_time(e1) / 5
    # the factors and the packed channel from one call (one launch at U = 32)
    fused = (fac, packed)
    api.factor_h16(H0, C, 1.0, out=fused)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(5):
        api.factor_h16(H0, C, 1.0, out=fused)
    e1.record()
    torch.cuda.synchronize()
    factor_pack_ms = e0.elapsed_time(e1) / 5
    for i in range(3):
        api.detect_factored_h16(packed, fac, frames[i % len(frames)][1], N0, B, U, C, 1.0, T, qam=qam, out=out)
    torch.cuda.synchronize()
    e0.record()
    for i in range(steps):
        api.detect_factored_h16(packed, fac, frames[i % len(frames)][1], N0, B, U, C, 1.0, T, qam=qam, out=out)
    e1.record()
    torch.cuda.synchronize()
    h16_ms = e0.elapsed_time(e1) / steps
    return {"factor_us_per_step": round(factor_ms * 1e3, 2), "detect_factored_us_per_step": round(det_ms * 1e3, 2),
            "detect_factored_vectors_per_s": round(n_sc / (det_ms * 1e-3), 1),
            "pack_h16_us_per_step": round(pack_ms * 1e3, 2),
            "factor_and_pack_h16_us_per_step": round(factor_pack_ms * 1e3, 2),
            "detect_h16_us_per_step": round(h16_ms * 1e3, 2),
            "detect_h16_vectors_per_s": round(n_sc / (h16_ms * 1e-3), 1),
            "note": "B_c^{-1} formed once per channel; each received frame runs the iterations only. h16: H resident "
                    "as complex FP16 with a power-of-two scale per (subcarrier, cluster), FP32 factors and iterations "
                    "(low-precision path, frame error <= 1e-3)"}


def reslice_cost(api, shapes=((256, 32, 8, 64, 0.0), (256, 32, 8, 64, 25.0), (512, 64, 8, 64, 0.0),
                                (128, 16, 8, 16, 0.0)), n_sc=1200, reps=20):
    """Cost of exact hard decisions: one 1200-subcarrier frame detected with
    and without hard decisions (the FP64 re-slice of near-threshold
    subcarriers), and how many subcarriers the FP64 pass recomputed."""
    import torch
    res = []
    for B, U, C, qam, snr in shapes:
        frames, N0 = make_frames(3, "admm", B, U, qam, snr, n_sc, seed=11)
        ws = _ws(api, n_sc, U, C)
        out = (torch.empty((n_sc, 1, U), dtype=torch.complex64, device="cuda"),
               torch.empty((n_sc, 1, U), dtype=torch.uint8, device="cuda"),
               torch.empty(n_sc, dtype=torch.int32, device="cuda"))
        t = {}
        for hard in (False, True):
            o = out if hard else (out[0], None, out[2])
            for i in range(3):
                api.detect(frames[i][0], frames[i][1], N0, C, 1.0, 5, qam=qam, out=o, workspace=ws, status=True)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for i in range(reps):
                api.detect(frames[i % 3][0], frames[i % 3][1], N0, C, 1.0, 5, qam=qam, out=o, workspace=ws,
                           status=True)
            e1.record()
            torch.cuda.synchronize()
            t[hard] = e0.elapsed_time(e1) / reps * 1e3
        n_res = int(((out[2] & 2) != 0).sum().item())
        res.append({"shape": f"B={B} U={U} C={C} {qam}-QAM {snr:g} dB", "n_sc": n_sc,
                    "us_soft_only": round(t[False], 1), "us_exact_hard": round(t[True], 1),
                    "resliced_subcarriers": n_res})
    return res


def copy_bandwidth_gbs(nbytes=1 << 30, reps=10):
    """Device-to-device copy rate measured on this GPU (read + write bytes per
    second), the STREAM-style reference for the kernels' HBM rates.  Kernels
    that mostly read can exceed it: a read-only stream avoids the bus
    turnarounds that an even mix of reads and writes pays."""
    import torch

    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def served_ratios(static, fp32_batched_us):
    """Vectors/s of the resident (served) forms relative to the plain FP32
    batched launch, when F received frames share one channel: per frame the
    channel's one-time work (factorisation, packing) is spread over F frames."""
    out = {}
    for name, once, per in (("fp32_resident", static["factor_us_per_step"], static["detect_factored_us_per_step"]),
                            ("h16_resident", static["factor_and_pack_h16_us_per_step"],
                             static["detect_h16_us_per_step"])):
        out[name] = {f"F={F}": round(fp32_batched_us / (once / F + per), 3) for F in (1, 7, 14, 70)}
        out[name]["F=inf"] = round(fp32_batched_us / per, 3)
    return out


def graph_small_frames(api, n_frames=16, reps=50):
    """Launch-bound small frames (B=64, U=8, C=4, 16 subcarriers, QPSK, T=3):
    n_frames detection calls issued eagerly against the same calls captured
    once in a HIP graph and replayed; microseconds per frame from events."""
    import torch

    B, U, C, n_sc, T = 64, 8, 4, 16, 3
    frames, N0 = make_frames(n_frames, "admm", B, U, 4, 10.0, n_sc, seed=99)
    outs = [(torch.empty((n_sc, 1, U), dtype=torch.complex64, device="cuda"),
             torch.empty((n_sc, 1, U), dtype=torch.uint8, device="cuda")) for _ in range(n_frames)]

    ws = api.workspace(n_sc, U, C)

    def body():
        for (H, y), o in zip(frames, outs):
            api.detect(H, y, N0, C, 1.0, T, qam=4, out=o, workspace=ws)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        body()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        body()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {}
    for name, fn in (("eager", body), ("graph", g.replay)):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        res[f"{name}_us_per_frame"] = round(e0.elapsed_time(e1) * 1e3 / (reps * n_frames), 2)
    res["frames_per_graph"] = n_frames
    res["shape"] = f"B={B} U={U} C={C} n_sc={n_sc} QPSK T={T}"
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="admm_ul_B256_U32_C8", choices=sorted(WORKLOADS))
    ap.add_argument("--frames", type=int, default=0, help="distinct resident frames (0: enough for >= 2 GB)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving (p50/p99) run")
    ap.add_argument("--no-compare", action="store_true", help="skip the mixed-precision comparison")
    ap.add_argument("--no-single-frame", action="store_true", help="skip the single-frame latency launches")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--frames-per-step", type=int, default=DEFAULT_FRAMES_PER_STEP,
                    help="1200-subcarrier frames processed by one launch (one step); 32 frames keep the "
                         "wave-scheduling tail of the launch near 1 %%")
    ap.add_argument("--n-sc", type=int, default=0, help="subcarriers per step (overrides --frames-per-step)")
    ap.add_argument("--T", type=int, default=0, help="override the iteration count of the workload")
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp16", "bf16"])
    ap.add_argument("--streams", type=int, default=1, help="streams that consecutive frames alternate over")
    ap.add_argument("--factor", default=None, choices=["auto", "fp32", "fp64", "f16x2"])
    ap.add_argument("--form", default="oneshot", choices=["oneshot", "resident", "resident_h16"],
                    help="oneshot: every step forms Gram and inverse (default); resident: a static channel's "
                         "factors (and for resident_h16 its FP16-packed H) are made once before timing and each "
                         "step runs the iterations for a new received frame")
    ap.add_argument("--serve-only", action="store_true", help="run only the serving benchmark")
    ap.add_argument("--serve-frames", type=int, default=10000, help="frames per offered load in the serving run")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="run only a plain device-to-device copy of this many bytes (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              f"(subcarriers shard across GPUs with no exchange: run one process per GPU on its share)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_bytes:
        src = torch.ones(args.copy_bytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(max(1, args.steps)):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_bytes, "launches": max(1, args.steps)}), flush=True)
        return

    from paper_1702_04458_amd import api

    if args.serve_only:
        print(json.dumps(serve_bench(frames_per_load=args.serve_frames)), flush=True)
        return

    algo, B, U, C, qam, snr, T, frame_sc = WORKLOADS[args.workload]
    n_sc = args.n_sc or frame_sc * args.frames_per_step
    if args.T:
        T = args.T
    if args.form != "oneshot":
        if algo != "admm" or args.prec != "fp32":
            print("--form resident* applies to the FP32 ADMM-UL workloads", file=sys.stderr)
            sys.exit(2)
        # the resident forms are measured on their own: no one-shot side legs
        args.no_compare = args.no_serve = args.no_single_frame = True
    bytes_vec = algorithmic_bytes(algo, B, U, C, args.form)
    flops_vec = algorithmic_flops(algo, B, U, C, T, args.form)
    frame_bytes = n_sc * (8 * B * U + 8 * B)
    n_frames = args.frames or max(2, math.ceil(2.0e9 / frame_bytes))
    print(f"[bench] {args.workload}: generating {n_frames} resident frames "
          f"({n_frames * frame_bytes / 1e9:.2f} GB)", file=sys.stderr, flush=True)
    frames, N0 = make_frames(n_frames, algo, B, U, qam, snr, n_sc, seed=1234)
    if algo == "dl":
        out = (torch.empty((n_sc, 1, B), dtype=torch.complex64, device="cuda"),
               torch.empty((n_sc, 1), dtype=torch.float32, device="cuda"))
    else:
        out = (torch.empty((n_sc, 1, U), dtype=torch.complex64, device="cuda"),
               torch.empty((n_sc, 1, U), dtype=torch.uint8, device="cuda"))
    resident = None
    if args.form != "oneshot":
        # frames received over one static channel (the channel whose factors are resident)
        H0 = frames[0][0]
        frames = [(H0, y) for y in received_over(H0, len(frames), qam, snr, seed=4321)]
        fac = api.factor(H0, C, 1.0)
        chan = H0 if args.form == "resident" else api.pack_channel_h16(H0, C)
        resident = (args.form, chan, fac, B, U)
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    ms_per_step, per = time_steps(api, frames, algo, C, T, N0, qam, out, args.prec, args.factor,
                                  args.steps, args.warmup, args.streams, resident)
    wall = time.perf_counter() - t0
    # The dominant kernel alone, for the roofline: the same launches without
    # hard decisions, so without the FP64 re-slice pass that follows the
    # kernel in the timed calls (the precoder and the FP16 channel have none).
    if algo == "dl" or args.form == "resident_h16":
        per_k = per
    else:
        _, per_k = time_steps(api, frames, algo, C, T, N0, qam, (out[0], None), args.prec, args.factor,
                              args.steps, args.warmup, 1, resident)
    avg_kernel_ms = sum(per_k) / len(per_k)
    vectors_per_s = n_sc / (ms_per_step * 1e-3)
    p50 = per[len(per) // 2]
    p99 = per[min(len(per) - 1, int(math.ceil(0.99 * len(per))) - 1)]
    print(f"[bench] timed {args.steps} steps: {ms_per_step * 1e3:.1f} us/step (wall {wall:.3f} s)",
          file=sys.stderr, flush=True)

    # single-frame launches (1200 subcarriers): per-frame latency of the batch form
    single = None
    if not args.no_single_frame:
        one = [(f[0][:frame_sc], f[1][:frame_sc]) for f in frames]
        one_out = tuple(t[:frame_sc] for t in out)
        one_ms, one_per = time_steps(api, one, algo, C, T, N0, qam, one_out, args.prec, args.factor, 50, 5)
        single = {"n_sc": frame_sc, "vectors_per_s": round(frame_sc / (one_ms * 1e-3), 1),
                  "p50_frame_latency_us": round(one_per[len(one_per) // 2] * 1e3, 2),
                  "p99_frame_latency_us": round(
                      one_per[min(len(one_per) - 1, int(math.ceil(0.99 * len(one_per))) - 1)] * 1e3, 2)}

    achieved_gbs = bytes_vec * n_sc / (avg_kernel_ms * 1e-3) / 1e9
    achieved_tflops = flops_vec * n_sc / (avg_kernel_ms * 1e-3) / 1e12
    hbm_floor = bytes_vec * n_sc / (HBM_PEAK_GBS * 1e9)
    alu_floor = flops_vec * n_sc / (FP32_VECTOR_PEAK_TFLOPS * 1e12)
    # the profiles are taken at the default step (DEFAULT_FRAMES_PER_STEP frames, FP32, workload T)
    profile_key = args.workload if args.form == "oneshot" else f"{args.workload}_{args.form}"
    traffic = (profiled_traffic(profile_key)
               if (args.prec == "fp32" and not args.n_sc and not args.T
                   and args.frames_per_step == DEFAULT_FRAMES_PER_STEP) else None)
    if alu_floor > hbm_floor:
        roof = {"bound": "alu", "achieved": round(achieved_tflops, 3), "peak": FP32_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved_tflops / FP32_VECTOR_PEAK_TFLOPS, 4), "traffic": traffic}
    else:
        roof = {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved_gbs / HBM_PEAK_GBS, 4), "traffic": traffic}
    roof["kernel_avg_us"] = round(avg_kernel_ms * 1e3, 2)
    roof["kernel_timing"] = ("HIP events around each launch of the dominant kernel alone (the same calls without "
                             "hard decisions, i.e. without the FP64 re-slice pass)")
    roof["hbm_achieved_gbs"] = round(achieved_gbs, 1)
    roof["hbm_frac"] = round(achieved_gbs / HBM_PEAK_GBS, 4)
    copy_gbs = copy_bandwidth_gbs()
    roof["measured_copy_gbs"] = round(copy_gbs, 1)
    roof["hbm_frac_of_measured_copy"] = round(achieved_gbs / copy_gbs, 4)
    roof["algorithmic_bytes_per_launch"] = bytes_vec * n_sc
    roof["algorithmic_flops_per_launch"] = flops_vec * n_sc

    compare = None
    if algo == "admm" and U == 32 and not args.no_compare:
        compare = {}
        for prec, factor in (("fp16", "auto"), ("fp16", "fp32"), ("fp16", "f16x2"), ("bf16", "auto"), ("bf16", "fp32"),
                             ("bf16", "f16x2")):
            ms, _ = time_steps(api, frames, algo, C, T, N0, qam, out, prec, factor, max(10, args.steps // 2), 3,
                               args.streams)
            compare[f"{prec}_factor_{factor}"] = {"vectors_per_s": round(n_sc / (ms * 1e-3), 1),
                                                  "us_per_step": round(ms * 1e3, 2)}
            print(f"[bench] mixed {prec} factor={factor}: {ms * 1e3:.1f} us/step", file=sys.stderr, flush=True)
        best = max(v["vectors_per_s"] for v in compare.values())
        compare["best_mixed_vs_fp32"] = round(best / vectors_per_s, 3)
        compare["rule_mixed_vs_fp32"] = round(compare["fp16_factor_auto"]["vectors_per_s"] / vectors_per_s, 3)
        compare["configuration_4"] = mixed_cfg4_bench(api)

    static = None
    if algo == "admm" and not args.no_compare:
        static = static_channel_bench(api, frames, C, T, N0, qam, snr, out, max(10, args.steps // 2))
        static["served_vs_fp32_batched"] = served_ratios(static, ms_per_step * 1e3)
        print(f"[bench] static channel: factor {static['factor_us_per_step']} us, factored detect "
              f"{static['detect_factored_us_per_step']} us/step, h16 detect {static['detect_h16_us_per_step']} us/step",
              file=sys.stderr, flush=True)

    graph = None
    if algo == "admm" and not args.no_compare:
        graph = graph_small_frames(api)
        print(f"[bench] small frames: eager {graph['eager_us_per_frame']} us, graph {graph['graph_us_per_frame']} us "
              f"per frame", file=sys.stderr, flush=True)

    serving = None
    if not args.no_serve and algo == "admm":
        print("[bench] serving run", file=sys.stderr, flush=True)
        serving = serve_bench(frames_per_load=args.serve_frames, pool=40)
        # the same mix without admission batching (one launch per frame)
        nb = serve_bench(loads=(0.85,), frames_per_load=max(1000, args.serve_frames // 5), pool=40, max_batch=1)
        serving["unbatched"] = {"saturation_fps": nb["saturation_fps"], "load_0.85": nb["loads"][0]}
        if U == 32 and args.form == "oneshot":
            serving["served_h16"] = serve_h16_bench(api, B=B, U=U, C=C, qam=qam, snr=snr)
            sat = serving["served_h16"]["saturation_vectors_per_s"]
            serving["served_h16"]["vs_fp32_batched"] = round(sat / vectors_per_s, 3)

    nsym7 = None
    reslice = None
    if algo == "admm" and not args.no_compare and args.form == "oneshot" and args.prec == "fp32":
        nsym7 = nsym_bench(api, B, U, C, qam, snr, T)
        reslice = reslice_cost(api)

    budget = None
    if algo == "dl" and not args.no_compare:
        budget = dl_budget_bench(api, frames, C, T, out, max(10, args.steps // 2))

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        cpu = cpu_baseline(algo, B, U, C, qam, snr, T, args.cpu_seconds)

    metric = "detected subcarrier-vectors/s at B=256,U=32 (mixed vs FP32) + p99 frame latency"
    dtype = {"fp32": "f32", "fp16": "f16+f32", "bf16": "bf16+f32"}[args.prec]
    if args.form == "resident_h16":
        dtype = "f16+f32"
    line = {
        "metric": metric,
        "value": round(vectors_per_s, 1),
        "unit": "vectors/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "algorithm": {"admm": "Algorithm 1 (ADMM-UL)", "cg": "Algorithm 2 (CG-UL)", "dl": "Algorithm 3 (ADMM-DL)"}[algo],
            "B": B, "U": U, "C": C, "S": B // C, "n_sc": n_sc, "n_sym": 1, "T": T, "rho": 1.0, "qam": qam,
            "snr_db": snr, "precision": args.prec, "factor": args.factor or "auto", "frames_resident": n_frames,
            "form": args.form,
            "step": f"one launch over {n_sc // frame_sc if n_sc % frame_sc == 0 else n_sc / frame_sc} frames "
                    f"of {frame_sc} subcarriers ({n_sc} subcarrier-vectors), inputs resident in HBM"
                    + ("" if args.form == "oneshot" else
                       "; detection against a static channel whose factors (resident_h16: and FP16-packed H) "
                       "were made once before timing"),
            "streams": args.streams,
            "p50_step_latency_us": round(p50 * 1e3, 2), "p99_step_latency_us": round(p99 * 1e3, 2),
            "single_frame": single,
            "mixed_precision": compare,
            "static_channel": static,
            "small_frames_graph": graph,
            "n_sym7": nsym7,
            "exact_hard_cost": reslice,
            "downlink_budgets": budget,
            "serving": serving,
        },
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
