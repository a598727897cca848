"""Write the stored oracle results of the long parity cases.

    python tests/golden/make_golden.py [name ...]

Every value written here comes from the FP64 CPU oracle (oracle/) run on the
seeded synthetic inputs of paper_1804_07135_amd.inputs; nothing is taken
from the HIP path.  The oracle follows Sec. II (eqs. (1)-(8), direct dipole
sum) and Sec. III (one descent step per iteration, eq. (10); arc-length
reparametrisation, eqs. (11)-(12)).  Runs too long to repeat inside a GPU
test (minutes on the host) are stored as JSON next to this script:

  boundary_64x64x1_k20.json   the 64x64x1 boundary-annihilation workload,
                              20 images, 200 iterations of step 0.1:
                              final energies, barrier, argmax, force norm,
                              and the final string at 4096 sampled entries
  sweep_points_100it.json     the (k_u, d) sweep's points of smallest and
                              largest lattice (L = 50 and 96), 16 images,
                              100 iterations of step 0.1: energies, barrier,
                              argmax, sampled string entries
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle  # noqa: E402
from paper_1804_07135_amd import inputs  # noqa: E402

N_SAMPLES = 4096


def sample_index(shape, seed=0):
    """Flat indices (sorted) of the sampled string entries."""
    n = int(np.prod(shape))
    return np.sort(np.random.default_rng(seed).choice(n, size=min(n, N_SAMPLES), replace=False))


def run_case(w, iters):
    s0 = inputs.build_string(w)
    t = time.time()
    r = oracle.iterate(s0, w["J"], w["d"], w["ku"], w["D"], iters, w["tau"])
    B, km = oracle.barrier(r["E"])
    # force norm of the final string (needs its fields)
    h = np.stack([oracle.field(si, w["J"], w["d"], w["ku"], w["D"]) for si in r["s"]])
    fn = oracle.force_norm(r["s"], h)
    idx = sample_index(r["s"].shape)
    out = {"workload": {k: v for k, v in w.items()}, "iters": iters, "E": r["E"].tolist(),
           "barrier": B, "argmax": km, "force_norm": fn, "sample_index": idx.tolist(),
           "sample_values": r["s"].ravel()[idx].tolist(), "oracle_seconds": time.time() - t}
    return out


def boundary():
    w = dict(inputs.WORKLOADS["boundary_64x64x1_k20"])
    return run_case(w, w["iters"])


def sweep_points():
    pts = inputs.sweep_points()
    Ls = [p["nx"] for p in pts]
    cases = []
    for i in (int(np.argmin(Ls)), int(np.argmax(Ls))):
        c = run_case(dict(pts[i]), 100)
        c["point"] = i
        cases.append(c)
    return {"points": cases}


CASES = {"boundary_64x64x1_k20": boundary, "sweep_points_100it": sweep_points}


def main(names):
    oracle.build()
    for name in names or list(CASES):
        data = CASES[name]()
        data["generator"] = "tests/golden/make_golden.py (oracle/ only)"
        with open(os.path.join(HERE, name + ".json"), "w") as fh:
            json.dump(data, fh)
        print(name, "written", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
