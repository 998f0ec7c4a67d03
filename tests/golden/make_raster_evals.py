"""Writes raster_evals_1080p_5p8m.json: the pixel-gaussian evaluations the
batched form needs on the benchmark workload (5.8M clustered gaussians,
1920x1080, orbit views 0, 10, ..., 50), counted by the oracle
(oracle.count_evals).  The benchmark divides the rasteriser's operation count
by its measured time with these figures.  Calls only the oracle and the
seeded scene generators.

  python tests/golden/make_raster_evals.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2606_00352_amd import scenes  # noqa: E402

VIEWS = (0, 10, 20, 30, 40, 50)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "raster_evals_1080p_5p8m.json")


def main():
    oracle.build()
    scene, cams = scenes.config1()
    rows = []
    for v in VIEWS:
        t0 = time.perf_counter()
        fr = oracle.frame(scene, cams[v], render=False)
        n_all, n_read = oracle.count_evals(fr.geo, fr.sorted_gid, fr.batch_tab, cams[v])
        rows.append({"view": v, "evals_all_units": n_all, "evals_merge_reads": n_read,
                     "pairs": int(fr.sorted_gid.shape[0]), "batches": int(fr.batch_tab.shape[0])})
        print(rows[-1], f"{time.perf_counter() - t0:.1f} s", flush=True)
    out = {"workload": "5.8M clustered gaussians (SH degree 3), 1920x1080, 60-view orbit, f=1100",
           "counted_by": "oracle.count_evals: 64 evaluations per gaussian whose level ellipse holds a "
                         "pixel centre of the render tile, until every pixel of the tile has local "
                         "T < t_eps; merge_reads: only (unit, tile) pairs whose partial the merge reads",
           "views": rows}
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
