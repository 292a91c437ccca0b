"""Writes the exact max-min fair allocations used as ground truth by the tests and the benchmark.

Inputs come from the seeded generators (``workloads``); the allocations come only from
``oracle.maxmin_exact`` (progressive filling of LPs, HiGHS).  Run from the repository root:

    python tests/golden/make_maxmin.py waxman20 waxman150 failures
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


def main(names):
    for name in names:
        if name == "failures":
            scenarios()
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
