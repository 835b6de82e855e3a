"""Write the stored expected values under tests/golden/ from the FP64 oracle only.

ialg_plain_1024.json: for the 1024x1024 workload (3 seeded c, max_iter 24, 512 march
steps, 10 bisection steps), the number of dual-quaternion updates the method runs
per frame (march samples through the first inside one, bisection, 6 normal samples,
each to escape or max_iter), plus hit counts. The benchmark divides this count by
the GPU time to report Julia iterations per second.

ialg_de_1024.json: the same for the same three frames marched by distance estimates
(at most 512 steps, hit below 1e-4, steps clamped to [1e-4, 0.25], 10 bisection steps
when a step lands inside).

ialg_voxel_1024.json: for the 1024^3 voxel grid (the paper's high-detail constant
PAPER_C[7] with its max_iter 15, identity slice), the updates classification runs
(escape index, or max_iter inside, summed over voxels) and the number of inside voxels.

ialg_project_512.json: for the three 512x512 projections (shadows) of the paper's
constants PAPER_C[7], [0], [4] (max_iter 15, 256 march steps, 10 bisection steps, 16
fibre offsets each), the updates the projection render runs: each march and bisection
sample tries its fibre points in order until one is inside; each of the 6 normal samples
runs all 16.

Run:  python tests/golden/make_golden.py [plain|de|voxel|project]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle      # noqa: E402
import workloads   # noqa: E402


def voxel():
    t = time.time()
    p, (nx, ny, nz) = workloads.voxel_1024()
    total, inside = 0, 0
    for k0 in range(0, nz, 64):   # slabs of 64 planes, to bound memory
        r = oracle.classify_grid(p, nx, ny, nz, voxels=_slab(nx, ny, k0, min(nz, k0 + 64)))
        total += r["total_iters"]
        inside += int(r["inside"].sum())
        print(k0, total, inside, flush=True)
    out = {"workload": "voxel_1024", "nx": nx, "ny": ny, "nz": nz, "max_iter": p.max_iter,
           "c": p.c, "total_iters": total, "inside": inside,
           "generator": "tests/golden/make_golden.py (FP64 oracle)",
           "oracle_seconds": round(time.time() - t, 1)}
    with open(os.path.join(HERE, "ialg_voxel_1024.json"), "w") as f:
        json.dump(out, f, indent=1)


def _slab(nx, ny, k0, k1):
    import numpy as np
    return np.arange(k0 * nx * ny, k1 * nx * ny, dtype=np.int64)


def project():
    t = time.time()
    frames = []
    for f, (ci, p) in enumerate(zip(workloads.PROJECT_C, workloads.project_512())):
        r = oracle.render(p)
        frames.append({"paper_c": ci, "c": p.c, "fibers": int(p.fiber.shape[0]),
                       "iters": r["total_iters"], "hits": int(r["mask"].sum())})
        print(frames[-1], flush=True)
    out = {"workload": "project_512", "width": 512, "height": 512, "max_iter": 15,
           "march_steps": 256, "bisect_steps": 10, "frames": frames,
           "total_iters": sum(f["iters"] for f in frames),
           "generator": "tests/golden/make_golden.py (FP64 oracle)",
           "oracle_seconds": round(time.time() - t, 1)}
    with open(os.path.join(HERE, "ialg_project_512.json"), "w") as fo:
        json.dump(out, fo, indent=1)


def main(which):
    if which == "voxel":
        return voxel()
    if which == "project":
        return project()
    frames = []
    t = time.time()
    ps = workloads.plain_1024() if which == "plain" else workloads.de_1024()
    for seed, p in zip((0, 1, 2), ps):
        r = oracle.render(p)
        frames.append({"seed": seed, "c": p.c, "iters": r["total_iters"],
                       "hits": int(r["mask"].sum())})
        print(frames[-1], flush=True)
    out = {"workload": f"{which}_1024", "width": 1024, "height": 1024, "max_iter": 24,
           "march_steps": 512, "bisect_steps": 10, "frames": frames,
           "total_iters": sum(f["iters"] for f in frames),
           "generator": "tests/golden/make_golden.py (FP64 oracle)",
           "oracle_seconds": round(time.time() - t, 1)}
    if which == "de":
        out.update({"march": "distance estimate", "de_hit_eps": ps[0].de_hit_eps,
                    "de_min_step": ps[0].de_min_step, "de_max_step": ps[0].de_max_step})
    with open(os.path.join(HERE, f"ialg_{which}_1024.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "plain")
