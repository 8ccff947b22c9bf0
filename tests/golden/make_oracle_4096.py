"""Write oracle_4096_stops.json: the CPU oracle's results for two 4096^2
stop-at-tolerance solves that take it minutes (the GPU tests compare against
these stored values instead of re-running the oracle).

  tol_1e-8  Laplace, boundary U[0,100] per edge node (seed 2), omega_opt(4096),
            stop when max |du| < 1e-8, checked every 10 iterations;
  paper     the paper's configuration (Sec. 2.1 and Sec. 4): north edge 1,
            other edges 0, omega 0.376, stop when max |du| < 1e-5, checked
            every 4000 iterations, at most 50000.

Stored per case: the stop iteration, the final change (exact bit pattern)
and the SHA-256 of the final n x n interior (float64, row-major), with a few
sampled cells.  Only oracle/ and the input generators are called.

    python tests/golden/make_oracle_4096.py [threads]
"""
import hashlib
import json
import os
import struct
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import laplace_random_boundary, laplace_top_edge  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_4096_stops.json")
SAMPLES = [(0, 0), (1, 4095), (2047, 2048), (4095, 0), (4095, 4095), (1000, 3000)]


def bits(x):
    return struct.unpack("<Q", struct.pack("<d", x))[0]


def case(name, g, omega, tol, max_iters, K, threads):
    t0 = time.time()
    r = oracle.sor_f64(g.u0, g.bdy, g.f, omega, tol, max_iters, K, threads=threads)
    return {"name": name, "n": g.n, "omega": omega, "tol": tol, "max_iters": max_iters,
            "check_every": K, "status": r.status, "iterations": r.iterations,
            "final_max_delta": r.final_max_delta,
            "final_max_delta_bits": f"{bits(r.final_max_delta):016x}",
            "u_sha256": hashlib.sha256(r.u.tobytes()).hexdigest(),
            "samples": [[i, j, f"{bits(float(r.u[i, j])):016x}"] for i, j in SAMPLES],
            "oracle_seconds": round(time.time() - t0, 1), "oracle_threads": threads}


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    g = laplace_random_boundary(4096, seed=2)
    out = {"citation": "Mittal 2014, Sec. 2.1 Eq. 1, Sec. 3.1, Algorithm 1; Sec. 4 (paper case)",
           "cases": [case("tol_1e-8", g, g.omega, 1e-8, 100000, 10, threads)]}
    print(json.dumps(out["cases"][-1]), flush=True)
    g = laplace_top_edge(4096, top=1.0)
    out["cases"].append(case("paper", g, 0.376, 1e-5, 50000, 4000, threads))
    print(json.dumps(out["cases"][-1]), flush=True)
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
