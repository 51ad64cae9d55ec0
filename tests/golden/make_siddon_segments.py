"""Write ``siddon_segments.json``: Siddon pieces per voxel-projection of the 512^3 / 360 / 512^2
workload, counted by the CPU oracle on a seeded sample of rays.

A piece is one non-empty segment between consecutive plane crossings of a ray inside the grid, so it
is one voxel read of the ray-driven projector (Section 2.1).  pieces per voxel-projection =
(mean pieces per ray) x Nu Nv / (Nx Ny Nz), because one projection holds Nu Nv rays.  This script calls
only the oracle; the stored value is the gather model's unit for the Siddon forward projector.

    python tests/golden/make_siddon_segments.py [n_rays]
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

OUT = os.path.join(HERE, "siddon_segments.json")
SEED = 20000


def count(n_rays: int, seed: int = SEED) -> dict:
    import oracle
    from paper_1905_03748_amd import inputs
    w = inputs.workload("medium")
    geo = oracle.Geometry.from_dict(w.geometry_dict())
    n_total = len(w.angles) * w.ndet[0] * w.ndet[1]
    idx = inputs.sample_indices(n_total, n_rays, seed)
    seg = oracle.siddon_segments(geo, w.angles, idx).astype(np.float64)
    scale = w.ndet[0] * w.ndet[1] / float(np.prod(w.nvox))
    return {"workload": "512^3 of 0.5 mm, 360 angles, 512^2 detector of 0.8 mm, DSO 1000, DSD 1500",
            "n_rays": int(n_rays), "seed": int(seed),
            "mean_pieces_per_ray": float(seg.mean()),
            "std_pieces_per_ray": float(seg.std(ddof=1)),
            "pieces_per_voxel_proj": float(seg.mean() * scale),
            "stderr_pieces_per_voxel_proj": float(seg.std(ddof=1) / np.sqrt(n_rays) * scale)}


if __name__ == "__main__":
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 200000
    rec = count(n)
    json.dump(rec, open(OUT, "w"), indent=1)
    print(json.dumps(rec))
