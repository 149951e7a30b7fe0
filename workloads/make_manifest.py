"""Write ``workloads/manifest.json``: the thresholds and edge counts the workloads use.

Run from the repository root: ``python -m workloads.make_manifest``.  Every
number it stores comes from the CPU oracle's threshold routine (eq. (cstar),
Section 2), so the GPU path never computes a size.
"""
from __future__ import annotations

import json
import os

from oracle import theory


def main() -> None:
    cs = {}
    for k, r in [(2, 3), (2, 4), (2, 5), (2, 6), (3, 3), (3, 4)]:
        c, x = theory.cstar(k, r)
        cs[f"{k},{r}"] = {"cstar": c, "xstar": x}
    n22 = 1 << 22
    c33 = cs["3,3"]["cstar"]
    doc = {
        "cstar": cs,
        "kcore_r3_k3_n4M": {
            "n": n22,
            "m_0.9cstar": int(round(0.9 * c33 * n22)),
            "m_1.1cstar": int(round(1.1 * c33 * n22)),
        },
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "manifest.json")
    with open(path, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
        f.write("\n")
    print(path)


if __name__ == "__main__":
    main()
