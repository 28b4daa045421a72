"""Write the stored oracle results used by the full-size GPU parity tests.

Calls only ``oracle/`` (and the seeded input generator).  For each workload it
stores the FP64 oracle's per-defect interaction energies, self terms and an
integer fingerprint of every footprint (count, sum of voxel ids, sum of squared
voxel ids), so the GPU rasteriser can be checked bit for bit without storing
the lists themselves.

Usage: python tests/golden/make_oracle_golden.py loops_128 mixed_256 paper_129
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import energy  # noqa: E402
from paper_2403_09158_amd import inputs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def fingerprint(fps):
    cnt = np.array([len(f) for f in fps], dtype=np.int64)
    s1 = np.array([int(np.sum(f.astype(np.int64))) for f in fps], dtype=np.int64)
    s2 = np.array([int(np.sum(f.astype(np.int64) ** 2)) for f in fps], dtype=np.int64)
    return cnt, s1, s2


def run(name):
    t = time.time()
    prob, defs = {
        "loops_128": lambda: inputs.loops_128(prec=0),
        "mixed_256": lambda: inputs.mixed_256(prec=0),
        "paper_129": lambda: inputs.paper_129(prec=0),
    }[name]()
    E, parts = energy.energies_fast(prob, defs, return_parts=True)
    cnt, s1, s2 = fingerprint(parts["fps"])
    out = os.path.join(HERE, f"oracle_{name}.npz")
    np.savez_compressed(out, E=E, B=parts["B"], count=cnt, idsum=s1, idsum2=s2, n=prob.n, ndef=len(defs))
    print(f"{name}: wrote {out} in {time.time() - t:.0f} s; |E| max {np.abs(E).max():.4g} eV", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or ["loops_128", "mixed_256", "paper_129"]:
        run(name)
