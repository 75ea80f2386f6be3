"""Writes fullsize_sha256.txt: SHA-256 digests of the oracle's states after a
few steps of the full-size workloads, so the GPU runs can be compared with
them bit for bit without storing gigabytes.  Calls only the oracle and the
seeded input generator; about 30 minutes on 8 host threads and 20 GB of
host memory.

    python tests/golden/make_fullsize_digests.py [name ...]

With names, only those cases are recomputed; the other lines are kept.
"""
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1711_06203_amd import workloads as W  # noqa: E402


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float64).tobytes()).hexdigest()


def cases():
    """name -> (problem, steps); the GPU test builds the same problems."""
    mol = W.kelvin_helmholtz(n=256, box=64)
    mol.scheme = 1
    return {
        "kh256_10": (W.kelvin_helmholtz(n=256, box=64), 10),
        "kh256_13species_1": (W.kelvin_helmholtz(n=256, box=64, nspec=13), 1),
        "kh256_mol2_2": (mol, 2),
        "cloud256_1": (W.cloud_wind(n=256, box=64, fine_box=32), 1),
        "two_clouds256_1": (W.two_clouds(n=256, box=64, fine_box=32), 1),
    }


def main(names=None):
    lines = ["# Oracle runs of the full-size workloads (see cases() in make_fullsize_digests.py):",
             "# name: dt of the last step (hex) / SHA-256 of the float64 C-order bytes of the level-0",
             "# state [/ of each fine patch's state, in patch order]."]
    path = os.path.join(HERE, "fullsize_sha256.txt")
    kept = {}
    if names and os.path.exists(path):
        for line in open(path):
            if ":" in line and not line.startswith("#"):
                kept[line.split(":", 1)[0].strip()] = line.rstrip("\n")
    for name, (prob, steps) in cases().items():
        if names and name not in names:
            if name in kept:
                lines.append(kept[name])
            continue
        if prob.fine_boxes:
            rc, rf, dts, cnt = oracle.run_two_level(prob, steps)
            states = [rc] + ([rf] if isinstance(rf, np.ndarray) else list(rf))
        else:
            U, dts, cnt = oracle.run_problem(prob, steps)
            states = [U]
        assert not np.asarray(cnt).any(), name
        lines.append(f"{name}: {float(dts[-1]).hex()} " + " ".join(digest(a) for a in states))
        print(lines[-1], flush=True)
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main(sys.argv[1:] or None)
