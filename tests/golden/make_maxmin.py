"""Writes the exact max-min fair allocations used as ground truth by the tests and the benchmark.

Inputs come from the seeded generators (``workloads``); the allocations come only from
``oracle.maxmin_exact`` (progressive filling of LPs, HiGHS).  Run from the repository root:

    python tests/golden/make_maxmin.py waxman20 waxman150 failures drift150
"""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

import oracle  # noqa: E402
import workloads  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def scenarios(n=512):
    """Exact max-min allocations of the n failure scenarios (seed 0) of the 20-node instance."""
    scen = workloads.failure_scenarios(0, n_scen=n)
    out = {}
    for i, inst in enumerate(scen):
        S, info = oracle.maxmin_exact(inst)
        out[f"S{i}"] = S
        out[f"fp{i}"] = np.array(inst.fingerprint())
        print(f"scenario {i}: {inst.summary()} {info}", flush=True)
    path = os.path.join(HERE, "maxmin_failures_s0.npz")
    np.savez_compressed(path, n=np.array(n), **out)
    print(f"wrote {path}", flush=True)


DRIFT_TIMES = [0.02, 0.05, 0.1, 0.3, 1.0, 3.0, 10.0, 30.0, 300.0]


def _drift_one(args):
    i, t = args
    inst = workloads.drift_path(workloads.waxman150(0), DRIFT_TIMES, seed=0)[i]
    S, info = oracle.maxmin_exact(inst)
    print(f"t = {t:g} s: {inst.summary()} cap_events={inst.meta['drift']['cap_events']} {info}", flush=True)
    return i, S, inst.fingerprint()


def drift150(workers=4):
    """Exact max-min allocations of the 150-node instance drifted along one sample path (seed 0,
    default drift parameters) to each of DRIFT_TIMES seconds after T_0."""
    from multiprocessing import Pool
    out = {"t": np.array(DRIFT_TIMES)}
    with Pool(workers) as pool:
        for i, S, fp in pool.imap_unordered(_drift_one, list(enumerate(DRIFT_TIMES))):
            out[f"S{i}"] = S
            out[f"fp{i}"] = np.array(fp)
    path = os.path.join(HERE, "maxmin_waxman150_drift_s0.npz")
    np.savez_compressed(path, **out)
    print(f"wrote {path}", flush=True)


def main(names):
    for name in names:
        if name == "failures":
            scenarios()
            continue
        if name == "drift150":
            drift150()
            continue
        inst = getattr(workloads, name)(0)
        print(inst.summary(), flush=True)
        S, info = oracle.maxmin_exact(inst, verbose=True)
        out = os.path.join(HERE, f"maxmin_{name}_s0.npz")
        np.savez_compressed(out, S=S, fingerprint=np.array(inst.fingerprint()), rounds=info["rounds"],
                            lps=info["lps"])
        print(f"wrote {out}: {info}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["waxman20", "waxman150"])
