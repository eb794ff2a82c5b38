"""Timings of the bandwidth sweep and the ragged batch on the GPU.

    python -m paper_2510_12705_amd.measure c4   # n = 16384, b = 16 .. 256, FP64 / FP32 / FP16 storage
    python -m paper_2510_12705_amd.measure c5   # 512 ragged FP32 bands: one batched call vs a loop
    python -m paper_2510_12705_amd.measure sigma  # sigma of the n = 32768 bidiagonal on the device
    python -m paper_2510_12705_amd.measure sym    # symmetric band -> tridiagonal, FP64 / FP32 storage
    python -m paper_2510_12705_amd.measure small  # n = 512, b = 32 and n = 8192, b = 64, N(0,1) bands
    python -m paper_2510_12705_amd.measure vectors  # reduction plus U and V (FP64), n = 8192 and 16384

Each case is timed as the best of two runs after one warm-up (host wall clock
around the call and a device synchronisation), in the default launch
configuration.  The roofline percentage divides the algorithmic bytes of the
reference tilewidth schedule (one 128-byte line of the storage type) by the
time and by MI355X's 8 TB/s.  Inputs come from ``inputs`` (synthetic, seeded).
"""
from __future__ import annotations

import sys
import time

import numpy as np

PEAK_BYTES_PER_S = 8.0e12
TW_REF = {8: 16, 4: 32, 2: 64}


def _best_ms(torch, fn, reps=2):
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t)
    return best * 1e3


def bandwidth_sweep(n=16384, bandwidths=(16, 32, 64, 128, 256)):
    import torch

    from . import bb, inputs
    bb.reset_params()
    for b in bandwidths:
        band = torch.from_numpy(inputs.band_uniform(n, b, inputs.seed_for_bandwidth_sweep(b))).cuda()
        out = []
        for dt, elem in ((torch.float64, 8), (torch.float32, 4), (torch.float16, 2)):
            t = band.to(dt)
            ms = _best_ms(torch, lambda: bb.bb_reduce(t, n, b))
            alg = bb.model_bytes(n, b, elem, TW_REF[elem])
            out.append("%s %.1f ms (%.1f%% roofline)" % (str(dt).split(".")[-1], ms,
                                                           100 * alg / (ms / 1e3) / PEAK_BYTES_PER_S))
        print("n=%d b=%d: %s" % (n, b, " | ".join(out)), flush=True)


def ragged_batch(count=512, seed=5):
    """The ragged batch as configured: the batched FP32 call with parameters from
    bb_autotune_batched, captured once into a hipGraph and replayed, against a
    loop of plain FP32 bb_reduce calls on one stream (and the untuned eager
    batched call for reference).  Replays are timed with events on the capture
    stream (median of 5 after a warm-up replay)."""
    import torch

    from . import bb, inputs
    bb.release()
    bb.reset_params()
    mats = inputs.ragged_batch(count=count, seed=seed)
    bands = [torch.from_numpy(np.ascontiguousarray(bd)).cuda().to(torch.float32) for (_, _, bd) in mats]
    ns = [m[0] for m in mats]
    bs = [m[1] for m in mats]
    ds = [torch.empty(max(x, 1), dtype=torch.float64, device="cuda") for x in ns]
    es = [torch.empty(max(x, 1), dtype=torch.float64, device="cuda") for x in ns]
    t_default = _best_ms(torch, lambda: bb.bb_reduce_batched(bands, ns, bs, ds=ds, es=es))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        p = bb.autotune_batched(ns, bs, bb.F32, stream=s)
        bb.bb_reduce_batched(bands, ns, bs, ds=ds, es=es, stream=s)   # plan for this stream, tuned
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    t_tuned_eager = _best_ms(torch, lambda: bb.bb_reduce_batched(bands, ns, bs, ds=ds, es=es, stream=s))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        bb.bb_reduce_batched(bands, ns, bs, ds=ds, es=es, stream=s)
    g.replay()
    torch.cuda.synchronize()
    assert bb.stream_status(s) == 0
    times = []
    for _ in range(5):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(s):   # replay() launches on the current stream
            e0.record()
            g.replay()
            e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    t_graph = float(np.median(times))
    bb.reset_params()

    def loop():
        for t, x, y, d, e in zip(bands, ns, bs, ds, es):
            bb.bb_reduce(t, x, y, d, e)

    t_loop = _best_ms(torch, loop)
    alg = sum(bb.model_bytes(x, y, 4, TW_REF[4]) for x, y in zip(ns, bs))
    print("%d ragged FP32 bands: graph replay of the autotuned batched call %.1f ms (%r); eager tuned %.1f ms, "
          "eager defaults %.1f ms; loop of single calls %.1f ms (%.2fx the graph replay); %.1f%% roofline" % (
              count, t_graph, p, t_tuned_eager, t_default, t_loop, t_loop / t_graph,
              100 * alg / (t_graph / 1e3) / PEAK_BYTES_PER_S), flush=True)
    bb.release()


def small_workloads(names=("n512_b32", "n8192_b64")):
    """The two smaller N(0,1) workloads (n = 512, b = 32 and n = 8192, b = 64), FP64 and
    FP32 storage, best of five after a warm-up."""
    import torch

    from . import bb, inputs
    bb.reset_params()
    for name in names:
        _, n, b, _, _ = inputs.WORKLOADS[name]
        band = torch.from_numpy(inputs.workload(name)).cuda()
        out = []
        for dt, elem in ((torch.float64, 8), (torch.float32, 4)):
            t = band.to(dt)
            ms = _best_ms(torch, lambda: bb.bb_reduce(t, n, b), reps=5)
            alg = bb.model_bytes(n, b, elem, TW_REF[elem])
            out.append("%s %.2f ms (%.1f%% roofline)" % (str(dt).split(".")[-1], ms,
                                                            100 * alg / (ms / 1e3) / PEAK_BYTES_PER_S))
        print("n=%d b=%d: %s" % (n, b, " | ".join(out)), flush=True)


def vectors(cases=("n8192_b64", "n16384_b128_uniform")):
    """bb_reduce_vectors (FP64; the reduction logs its reflectors, U and V are
    formed from the identity, stage by stage beside the reduction) against
    bb_reduce alone on the same band; the difference is the time the
    back-transformation adds.  Its arithmetic: every reflector of a stage meets
    every row of its factor once, a dot and an update of its m + 1 entries
    (4 (m + 1) flops), counted over that added time."""
    import torch

    from . import bb, inputs
    bb.reset_params()
    for name in cases:
        _, n, b, _, _ = inputs.WORKLOADS[name]
        band = torch.from_numpy(inputs.workload(name)).cuda()
        t_red = _best_ms(torch, lambda: bb.bb_reduce(band, n, b))
        t_vec = _best_ms(torch, lambda: bb.bb_reduce_vectors(band, n, b))
        flops = 0.0
        tw = 32
        bs = b
        while bs > 1:
            t = min(tw, bs - 1)
            c = bs - t
            for r in range(0, n - c - 1):
                steps = 1 + (n - 2 - r - c) // bs
                # step 0 has m = b - c = t entries past the first; later steps min(t, n - 1 - p)
                flops += 2 * steps * n * 4 * (t + 1)
            bs = c
        back_ms = t_vec - t_red
        print("n=%d b=%d: reduction %.1f ms, with U and V %.1f ms (added %.1f ms, %.0f GFLOP/s over it)" % (
            n, b, t_red, t_vec, back_ms, flops / (back_ms / 1e3) / 1e9), flush=True)
        del band
        torch.cuda.empty_cache()


def symmetric(cases=((8192, 64), (32768, 128))):
    """The symmetric band -> tridiagonal reduction (bb_sym_reduce), FP64 and FP32
    storage, N(0,1) lower bands: time and % of roofline by the symmetric
    algorithmic bytes at the one-cache-line tilewidth."""
    import torch

    from . import bb
    bb.reset_params()
    for n, b in cases:
        rng = np.random.default_rng(n + b)
        band = torch.from_numpy(rng.standard_normal((n, b + 1))).cuda()
        out = []
        for dt, elem in ((torch.float64, 8), (torch.float32, 4)):
            t = band.to(dt)
            ms = _best_ms(torch, lambda: bb.bb_sym_reduce(t, n, b))
            alg = bb.sym_model_bytes(n, b, elem, TW_REF[elem])
            out.append("%s %.1f ms (%.1f%% roofline)" % (str(dt).split(".")[-1], ms,
                                                           100 * alg / (ms / 1e3) / PEAK_BYTES_PER_S))
        print("symmetric n=%d b=%d: %s" % (n, b, " | ".join(out)), flush=True)


def bidiag_sigma(n=32768, b=128):
    """sigma of the bidiagonal that the n = 32768, b = 128 reduction returns: the device
    bisection (bb_bidiag_sigma) against LAPACK dsterf on the host (one core), the
    routine the CPU reference uses on the same Golub-Kahan tridiagonal."""
    import torch

    from . import bb, inputs
    bb.reset_params()
    band = torch.from_numpy(inputs.workload("n%d_b%d" % (n, b))).cuda()
    d, e = bb.bb_reduce(band, n, b)
    torch.cuda.synchronize()
    ms = _best_ms(torch, lambda: bb.bidiag_sigma(d, e))
    sig = bb.bidiag_sigma(d, e).cpu().numpy()
    from scipy.linalg import lapack
    off = np.zeros(2 * n - 1)
    off[0::2] = d.cpu().numpy()
    off[1::2] = e.cpu().numpy()[: n - 1]
    t = time.perf_counter()
    w, info = lapack.dsterf(np.zeros(2 * n), off)
    host_ms = (time.perf_counter() - t) * 1e3
    ref = np.sort(w)[::-1][:n].clip(min=0.0)
    # Sturm-count work: the coarse pass counts at 4n points; then value j takes
    # ceil(log_9(cell / max(4 eps sigma_j, 2^-60 hi0))) steps of 8 counts from its
    # cell (width hi0 / 3n); a count is 2n - 1 steps of one multiply and one
    # multiply-add per point plus the shared square of the entry (about 4 flops)
    off_abs = np.abs(off)
    hi0 = np.max(np.concatenate([off_abs[:1], off_abs[1:] + off_abs[:-1], off_abs[-1:]])) * (1 + 4 * 2.0 ** -52)
    stop = np.maximum(4 * 2.0 ** -52 * sig, 2.0 ** -60 * hi0)
    iters = np.maximum(np.ceil(np.log((hi0 / (3 * n)) / stop) / np.log(9.0)), 0)
    counts = 4.0 * n + 8.0 * float(np.sum(iters))
    flops = counts * (2 * n - 1) * 4
    print("n=%d: device multisection %.1f ms (%.0f GFLOP/s of Sturm counts), host dsterf %.1f ms (%.0fx); "
          "max |sigma_dev - sigma_dsterf| / sigma_max = %.2e" % (
              n, ms, flops / (ms / 1e3) / 1e9, host_ms, host_ms / ms, np.max(np.abs(sig - ref)) / ref[0]),
          flush=True)


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "c4"
    {"c4": bandwidth_sweep, "c5": ragged_batch, "sigma": bidiag_sigma, "sym": symmetric,
     "small": small_workloads, "vectors": vectors}[what]()
