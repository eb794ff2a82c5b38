"""Write the full-size expected values that the GPU parity tests and bench.py check.

Every value here comes from the CPU oracle (``oracle/``) run on the seeded
synthetic inputs of ``paper_2510_12705_amd.inputs`` -- nothing is taken from
the GPU library.  The oracle takes minutes at these sizes, so the tests read
the stored results instead of recomputing them.

    python tests/golden/make_golden.py [--jobs 8] [--only NAME ...]

Outputs (in this directory):
  * ``full_size.json``: per entry the workload, the storage type whose
    rounding was applied to the FP64 draws before the FP64 oracle ran, the
    inner tilewidth TW, the SHA-256 of the oracle's d bytes followed by its e
    bytes (float64, little endian), a few scalars for diagnostics, and the name
    of the sigma file if one was written;
  * ``sigma_<entry>.npy``: the oracle's singular values (descending float64,
    LAPACK dsterf on the Golub-Kahan tridiagonal of the oracle's (d, e)).

Entries (workloads as in the input recipe; the paper's accuracy method,
Sec. V-A, compares against an FP64 reference of the same matrix):
  * n = 32768, b = 128, N(0,1): FP64 at TW 16 and 32 (hash); sigma of the FP64
    input and of its FP32 rounding;
  * n = 16384, b in {16, 32, 64, 128, 256}, U[-1,1]: FP64 at TW 32 (hash);
    sigma of the FP64 input and of its FP32 and FP16 roundings.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def entries():
    out = []
    for tw in (16, 32):
        out.append(dict(name="n32768_b128_f64_tw%d" % tw, workload="n32768_b128", rounding="f64", tw=tw,
                        sigma=(tw == 32)))
    out.append(dict(name="n32768_b128_f32_tw32", workload="n32768_b128", rounding="f32", tw=32, sigma=True))
    for b in (16, 32, 64, 128, 256):
        w = "n16384_b%d_uniform" % b
        out.append(dict(name="%s_f64_tw32" % w, workload=w, rounding="f64", tw=32, sigma=True))
        out.append(dict(name="%s_f32_tw32" % w, workload=w, rounding="f32", tw=32, sigma=True))
        out.append(dict(name="%s_f16_tw32" % w, workload=w, rounding="f16", tw=32, sigma=True))
    return out


def de_hash(d, e) -> str:
    import numpy as np
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(d, dtype="<f8").tobytes())
    h.update(np.ascontiguousarray(e, dtype="<f8").tobytes())
    return h.hexdigest()


def rounded(band, rounding):
    import numpy as np
    if rounding == "f64":
        return band
    dt = {"f32": np.float32, "f16": np.float16}[rounding]
    return band.astype(dt).astype(np.float64)


def run(ent):
    import numpy as np

    import oracle
    from paper_2510_12705_amd import inputs
    _, n, b, _, _ = inputs.WORKLOADS[ent["workload"]]
    band = rounded(inputs.workload(ent["workload"]), ent["rounding"])
    t0 = time.perf_counter()
    d, e = oracle.reduce(band, n, b, ent["tw"])
    t_red = time.perf_counter() - t0
    rec = dict(ent)
    rec.update(n=n, b=b, de_sha256=de_hash(d, e), d0=float(d[0]), abs_e0=float(abs(e[0])),
               sum_d2_e2=float(np.sum(d * d) + np.sum(e * e)), oracle_seconds=round(t_red, 2))
    if ent["sigma"]:
        s = oracle.singular_values(d, e)
        fn = "sigma_%s.npy" % ent["name"]
        np.save(os.path.join(HERE, fn), s, allow_pickle=False)
        rec.update(sigma_file=fn, sigma_max=float(s[0]), sigma_min=float(s[-1]))
    else:
        rec.update(sigma_file=None)
    del rec["sigma"]
    print("%s: oracle %.1f s" % (ent["name"], t_red), flush=True)
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", nargs="*")
    args = ap.parse_args()
    import oracle
    oracle.build(force=False)
    todo = [x for x in entries() if not args.only or x["name"] in args.only]
    # longest first
    todo.sort(key=lambda x: (x["workload"] != "n32768_b128", "b256" not in x["workload"]))
    path = os.path.join(HERE, "full_size.json")
    old = {}
    if os.path.exists(path):
        with open(path) as f:
            old = {r["name"]: r for r in json.load(f)["entries"]}
    with ProcessPoolExecutor(max_workers=args.jobs) as ex:
        for rec in ex.map(run, todo):
            old[rec["name"]] = rec
    order = [x["name"] for x in entries()]
    out = {"generator": "tests/golden/make_golden.py (CPU oracle only)",
           "hash": "SHA-256 of d then e as little-endian float64",
           "entries": [old[k] for k in order if k in old]}
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
