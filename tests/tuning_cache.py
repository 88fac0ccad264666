"""The launch tuning bench.py uses for a workload, read from the autotuner's
cache committed with the package."""


def bench_tuning(scene, lights, ppl, B):
    """The launch tuning bench.py uses for this workload (the autotuner's cache
    entry), or None."""
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2310_02043_amd",
                        "tuning.cache")
    want = (f"tris={scene.n_tris} texels={scene.n_texels} lights={lights.n_lights} layouts={lights.n_layouts} "
            f"ppl={ppl} hits={B}")
    best = None
    for line in open(path):
        key, _, vals = line.strip().partition("|")
        if key.endswith(want):
            v = vals.split()
            best = dict(zip(("waves_per_block", "xcd_remap", "tile_paths", "refill_threshold", "lds_depth",
                             "tri_share"), (int(x) for x in v[:6])))
    return best
