"""Write stored oracle values for a named workload (default: the 12,288-atom water box), one seed.

Calls only the FP64 oracle (oracle/) on inputs from the seeded generator.  The GPU
tests compare the library's set-up and steps with these values, and the benchmark
states its energy error against them, because the oracle needs half a minute or
more per step at this size.  Each step also records the oracle's count of the
algorithmic work of its passes (orc_work), which the library's own counters are
checked against.

    python tests/golden/make_golden.py [n_steps] [seed] [config]

The options a workload needs besides its system (synth.RUN_OPTIONS: the charge term) apply to the
oracle too; the tile capacity is a library option and has no counterpart there.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle.oracle import Oracle  # noqa: E402
from paper_1402_2880_amd import synth  # noqa: E402


def main(n_steps: int = 25, seed: int = 1, config: str = "water4096"):
    s = synth.make_config(config, seed)
    t = time.time()
    opts = {k: v for k, v in synth.RUN_OPTIONS.get(config, {}).items() if k == "scc"}
    o = Oracle(s, eps=1e-5, e_conv=1e-6, **opts)
    o.set_count(True)
    init = o.init_info()
    sample = np.arange(0, s.n_atoms, 97)
    rec = dict(config=config, seed=seed, eps=1e-5, e_conv=1e-6, n_atoms=s.n_atoms, n_ao=s.n_ao, options=opts,
               init=dict(energy=init["energy"], n_ortho_sweeps=init["n_ortho_sweeps"],
                         charges_sample=o.charges()[sample].tolist()),
               charge_sample_atoms=sample.tolist(), steps=[])
    print("init", round(time.time() - t, 1), init["energy"], flush=True)
    for k in range(n_steps):
        t = time.time()
        si = o.step()
        rec["steps"].append(dict(energy=si["energy"], delta_e=si["delta_e"], dq_max=si["dq_max"],
                                 n_candidates=si["n_candidates"], n_rotations=si["n_rotations"],
                                 n_ortho_sweeps=si["n_ortho_sweeps"], converged=si["converged"],
                                 post_ortho=si["post_ortho"], max_abs_fov=si["max_abs_fov"],
                                 nnz_c=si["nnz_c"], work=o.work(),
                                 charges_sample=o.charges()[sample].tolist()))
        print("step", k + 1, round(time.time() - t, 1), si["energy"], flush=True)
        # written after every step, so that an interrupted run keeps what it has
        out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{config}_seed{seed}.json")
        with open(out + ".tmp", "w") as f:
            json.dump(rec, f, indent=1)
        os.replace(out + ".tmp", out)
    print("wrote", out)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 25, int(sys.argv[2]) if len(sys.argv) > 2 else 1,
         sys.argv[3] if len(sys.argv) > 3 else "water4096")
