"""Writes tests/golden/oracle_solves.json: iteration counts and residuals of
the CPU oracle for the benchmark's configurations.  Calls only oracle/ and
the seeded input generators."""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2507_11512_amd import inputs  # noqa: E402

CASES = [
    # name, dims, levels, sweep, x0 kind
    ("tiny_16_sym", (16, 16, 16), 3, 2, "zero"),
    ("fwd_32", (32, 32, 32), 4, 0, "zero"),
    ("fwd_64", (64, 64, 64), 4, 0, "zero"),
    ("mid_128", (128, 128, 128), 4, 0, "zero"),
    ("mid_128_random_x0", (128, 128, 128), 4, 0, "random"),
]


def sample_rows(n, count=1024, seed=11512):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([rng.integers(0, n, count), [0, n - 1]]))


def main():
    out = {"note": "oracle FP64 (f32=false) and FP32-storage emulation (f32=true) solves, "
                   "b = A*1, GMRES(30), tol 1e-9, beta = 0.5, 1/1/1 sweeps",
           "cases": {}}
    for name, dims, levels, sweep, x0k in CASES:
        b = oracle.spmv(dims, inputs.ones(dims))
        x0 = inputs.random_x0(dims) if x0k == "random" else None
        rec = {"dims": dims, "levels": levels, "sweep": sweep, "x0": x0k}
        for f32 in (False, True):
            t = time.time()
            x, st = oracle.gmres_ir(dims, b, x0=x0, levels=levels, sweep=sweep, restart=30,
                                    tol=1e-9, f32=f32)
            key = "f32" if f32 else "f64"
            rec[key] = {"iters": st.iters, "restarts": st.restarts,
                        "final_rel_res": st.final_rel_res,
                        "x_err_vs_ones": float(np.linalg.norm(x - 1) / np.sqrt(x.size)),
                        "x_norm": float(np.linalg.norm(x))}
            if x.size >= 128 ** 3 and not f32:
                # sampled entries of the oracle's solution, for parity of x at
                # sizes where the test cannot rerun the oracle solve
                rows = sample_rows(x.size)
                rec[key]["sample_rows"] = rows.tolist()
                rec[key]["sample_x"] = [float(v) for v in x[rows]]
            print(name, key, {k: v for k, v in rec[key].items() if not k.startswith("sample")},
                  f"{time.time() - t:.1f}s", flush=True)
        out["cases"][name] = rec
    with open(os.path.join(HERE, "oracle_solves.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
