"""Write oracle reference results for the parity tests (calls only oracle/ and workload/).

    python tests/golden/make_golden.py mid            # N = 6000, energies 0, 9, 19
    python tests/golden/make_golden.py large 0        # N = 25600, energy 0 (hours of CPU)

Output: tests/golden/<config>_oracle.npz with, per energy index e, arrays
E_e, R_e, S_e (complex128) and sigma_e, plus the oracle thread count.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ge, pipeline, system  # noqa: E402
from workload import make_system  # noqa: E402

DEFAULT_ENERGIES = {"small": list(range(10)), "mid": [0, 9, 19], "large": [0]}


def main(argv):
    config = argv[1] if len(argv) > 1 else "mid"
    idx = [int(x) for x in argv[2:]] or DEFAULT_ENERGIES[config]
    ge.build(force=False)
    sp = make_system(config)
    md = system.MeshData(sp.nr, sp.a)
    out_path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{config}_oracle.npz")
    data = dict(np.load(out_path)) if os.path.exists(out_path) else {}
    data["threads"] = np.array(ge.threads())
    for e in idx:
        E = float(sp.energies[e])
        t0 = time.time()
        o = pipeline.solve_energy(sp, E, md)
        data[f"E_{e}"] = np.array(E)
        data[f"R_{e}"] = o["R"]
        data[f"S_{e}"] = o["S"]
        data[f"sigma_{e}"] = o["sigma"]
        print(f"{config} energy {e} E={E:.4f} done in {time.time() - t0:.1f} s", flush=True)
        np.savez_compressed(out_path, **data)
    print("wrote", out_path)


if __name__ == "__main__":
    main(sys.argv)
