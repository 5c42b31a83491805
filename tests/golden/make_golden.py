"""Write oracle reference results for the parity tests (calls only oracle/ and workload/).

    python tests/golden/make_golden.py mid            # N = 6000, energies 0, 9, 19
    python tests/golden/make_golden.py large 0        # N = 25600, energy 0 (hours of CPU)
    python tests/golden/make_golden.py mid --floor    # also the FP64 floor (see below)

Output: tests/golden/<config>_oracle.npz with, per energy index e, arrays
E_e, R_e, S_e (complex128) and sigma_e, plus the oracle thread count.

FP64 floor: the same physical system with its channels numbered in reverse
order is an equivalent linear system whose elimination rounds differently.
Its R and S, mapped back, differ from the first solve only by FP64 rounding
amplified by the conditioning of the system; Rfloor_e and Sfloor_e store that
difference (max|x - ref| / max|ref|), the accuracy to which FP64 arithmetic
determines R and S at all.
"""
from __future__ import annotations

import copy
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ge, pipeline, system  # noqa: E402
from workload import make_system  # noqa: E402

DEFAULT_ENERGIES = {"small": list(range(10)), "mid": [0, 9, 19], "large": [0]}


def reversed_channels(sp):
    rv = copy.deepcopy(sp)
    rv.l = sp.l[::-1].copy()
    rv.eps = sp.eps[::-1].copy()
    rv.beta = sp.beta[::-1, ::-1].copy()
    return rv


def save(path, data):
    tmp = path + ".tmp.npz"
    np.savez_compressed(tmp, **data)
    os.replace(tmp, path)


def relerr(x, ref):
    return float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))


def main(argv):
    args = [a for a in argv[1:] if not a.startswith("--")]
    floor = "--floor" in argv
    config = args[0] if args else "mid"
    idx = [int(x) for x in args[1:]] or DEFAULT_ENERGIES[config]
    ge.build(force=False)
    sp = make_system(config)
    md = system.MeshData(sp.nr, sp.a)
    out_path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{config}_oracle.npz")
    data = dict(np.load(out_path)) if os.path.exists(out_path) else {}
    data["threads"] = np.array(ge.threads())
    for e in idx:
        E = float(sp.energies[e])
        if f"S_{e}" not in data:
            t0 = time.time()
            o = pipeline.solve_energy(sp, E, md)
            data[f"E_{e}"] = np.array(E)
            data[f"R_{e}"] = o["R"]
            data[f"S_{e}"] = o["S"]
            data[f"sigma_{e}"] = o["sigma"]
            print(f"{config} energy {e} E={E:.4f} done in {time.time() - t0:.1f} s", flush=True)
            save(out_path, data)
        if floor and f"Rfloor_{e}" not in data:
            t0 = time.time()
            o2 = pipeline.solve_energy(reversed_channels(sp), E, md)
            data[f"Rfloor_{e}"] = np.array(relerr(o2["R"][::-1, ::-1], data[f"R_{e}"]))
            data[f"Sfloor_{e}"] = np.array(relerr(o2["S"][::-1, ::-1], data[f"S_{e}"]))
            print(f"{config} energy {e} floor R {float(data[f'Rfloor_{e}']):.2e} "
                  f"S {float(data[f'Sfloor_{e}']):.2e} in {time.time() - t0:.1f} s", flush=True)
            save(out_path, data)
    print("wrote", out_path)


if __name__ == "__main__":
    main(sys.argv)
