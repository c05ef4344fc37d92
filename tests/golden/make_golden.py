"""Write the oracle's reference outputs for the small workload.

Calls only the CPU oracle and the seeded input generator.  The paper prints no
numeric worked example (its results are figures and timing tables), so the
stored values here are the oracle's own, kept as a regression anchor for the
oracle and as expected values for the GPU parity tests.

Usage: python tests/golden/make_golden.py
"""
import hashlib
import json
import math
import sys
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

import oracle  # noqa: E402
from paper_2506_11547_amd import datagen  # noqa: E402


def record(name: str) -> dict:
    w, inst = datagen.make_workload(name)
    r = oracle.get().solve(inst.x, inst.y, w.grid, w.samples, math.radians(w.eps_deg), w.topk)
    return {
        "workload": name,
        "cite": "Alg. 1 (voting) and Sec. 4.4 (several peaks), rescored with App. D's constraint",
        "n": w.n, "grid": w.grid, "samples": w.samples, "eps_deg": w.eps_deg, "topk": w.topk,
        "seed": w.seed,
        "input_sha256": hashlib.sha256(inst.x.tobytes() + inst.y.tobytes()).hexdigest(),
        "hist_sha256": hashlib.sha256(r["hist"].tobytes()).hexdigest(),
        "hist_sum": int(r["hist"].sum()),
        "hist_nonzero": int(np.count_nonzero(r["hist"])),
        "top_counts": r["top_counts"].tolist(),
        "top_idx": r["top_idx"].tolist(),
        "cand_counts": r["cand_counts"].tolist(),
        "winner": r["winner"],
        "q_bits": [int(b) for b in r["q"].view(np.uint32)],
        "count": r["count"],
        "mask_sha256": hashlib.sha256(r["mask"].astype(np.uint8).tobytes()).hexdigest(),
    }


if __name__ == "__main__":
    out = Path(__file__).resolve().parent / "small_oracle.json"
    out.write_text(json.dumps(record("small"), indent=1) + "\n")
    print("wrote", out)
