"""Writes the stored oracle outputs under tests/golden/.  Calls only the oracle and the seeded
input module; run from the repository root:  python tests/golden/make_golden.py"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import vdwdf  # noqa: E402
from paper_1703_06999_amd import inputs  # noqa: E402


def hello_world():
    grid, cell, n, s = inputs.hello_world_inputs()
    kt = inputs.synthetic_kernel_table()
    E, dn, ds = vdwdf.energy_and_partials(n, s, cell, kt)
    return {
        "citation": "libvdwxc paper, Sec. 6 (The library): minimal example program; the paper "
                    "prints the inputs but not the resulting energy",
        "input": {"grid": list(grid), "cell": cell.tolist(), "rho": n.ravel().tolist(),
                  "sigma": s.ravel().tolist(), "functional": "vdW-DF1"},
        "synthetic_table": {"energy": E, "dedrho": dn.ravel().tolist(), "dedsigma": ds.ravel().tolist(),
                            "note": "oracle output with the synthetic Gaussian kernel table"},
    }


if __name__ == "__main__":
    with open(os.path.join(HERE, "hello_world.json"), "w") as f:
        json.dump(hello_world(), f, indent=1)
        f.write("\n")
