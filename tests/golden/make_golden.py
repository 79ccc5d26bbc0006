"""Write the stored FP64-oracle results that the GPU tests and the benchmark
compare against, for workloads too large to run the oracle inside a test.

Every value here comes from the plain FP64 oracle (``oracle/pogs_oracle.py``)
on the seeded inputs of ``paper_1503_08366_amd/workloads.py``; nothing is read
from the GPU library.  Each record carries the fingerprint of the inputs it
was computed on (``workloads.fingerprint``), so a change to a generator makes
the record unusable instead of silently wrong.

    python tests/golden/make_golden.py dose|batch|path|lasso [--jobs N]

Parameters are those of the workloads themselves (eps_abs 1e-4, eps_rel 1e-3,
the workload's iteration cap) with the float32 machine epsilon in the
equilibration's gamma (the GPU iterates on float32 matrices), the oracle's
defaults otherwise (Section 5: alpha 1.7, delta 1.05, tau 0.8, rho0 1).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FLT_EPS = float(np.finfo(np.float32).eps)


def _solve(p):
    from oracle import pogs_oracle as O
    prm = O.Params(eps_abs=p.eps_abs, eps_rel=p.eps_rel, max_iter=p.max_iter, eps_cmp=FLT_EPS)
    t = time.perf_counter()
    r = O.solve(p.A.astype(np.float64), p.f, p.g, prm)
    return {"optval": float(r.optval), "iters": int(r.iters), "converged": bool(r.converged),
            "r_pri": float(r.r_pri), "r_dual": float(r.r_dual), "seconds": time.perf_counter() - t}


def _batch_one(i):
    from paper_1503_08366_amd import workloads as W
    p = W.batch_member(i)
    rec = _solve(p)
    rec.update({"index": i, "kind": p.name, "m": p.m, "n": p.n, "fingerprint": W.fingerprint(p)})
    return rec


def _write(name, payload):
    """JSON with one result record per line."""
    path = os.path.join(HERE, name)
    recs = payload.pop("results")
    with open(path, "w") as fh:
        fh.write("{\n")
        for k, v in payload.items():
            fh.write(f" {json.dumps(k)}: {json.dumps(v)},\n")
        fh.write(' "results": [\n' + ",\n".join("  " + json.dumps(r) for r in recs) + "\n ]\n}\n")
    print(f"wrote {path}", flush=True)


def main():
    from paper_1503_08366_amd import workloads as W
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["dose", "batch", "path", "lasso"])
    ap.add_argument("--jobs", type=int, default=8)
    args = ap.parse_args()
    common = {"source": "FP64 oracle (oracle/pogs_oracle.py), eps_cmp = float32 machine epsilon",
              "numpy": np.__version__}
    if args.what == "dose":
        p = W.dose_100000x1000()
        rec = _solve(p)
        rec.update({"workload": "dose_100000x1000 (seed 2)", "fingerprint": W.fingerprint(p),
                    "objective_constant": float(p.f.const)})
        _write("dose_100000x1000.json", {**common, "results": [rec]})
    elif args.what == "lasso":
        out = []
        for name in ("lasso_20000x2000", "nnls_20000x2000"):
            p = getattr(W, name)()
            rec = _solve(p)
            rec.update({"workload": name, "fingerprint": W.fingerprint(p)})
            out.append(rec)
            print(name, rec, flush=True)
        _write("lasso_20000x2000.json", {**common, "results": out})
    elif args.what == "path":
        probs = W.lambda_path()
        out = []
        for r, p in enumerate(probs):
            rec = _solve(p)
            rec.update({"r": r, "lam": p.meta["lam"], "fingerprint": W.fingerprint(p)})
            out.append(rec)
            print(r, rec["iters"], rec["optval"], flush=True)
        _write("lambda_path_8000x1000.json", {**common, "workload": "lambda_path (seed 33, R 64)", "results": out})
    else:
        import multiprocessing as mp
        for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            os.environ[k] = "1"
        with mp.get_context("spawn").Pool(args.jobs) as pool:
            out = []
            for rec in pool.imap(_batch_one, range(512), chunksize=4):
                out.append(rec)
                if len(out) % 32 == 0:
                    print(f"{len(out)}/512", flush=True)
        _write("batch_mix_512.json", {**common, "workload": "batch_mix (seed 3, 512 problems)", "results": out})


if __name__ == "__main__":
    main()
