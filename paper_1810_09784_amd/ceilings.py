"""Measured ceilings of the GPU: runs the microbenchmark that build() compiles
from csrc/ceilings.hip (FP64 fma and fma + cvt, LDS atomic adds by access
pattern, HBM read / copy / store, dense BF16 MFMA) and stores its results
beside this module, where bench.py reads them to put its rooflines next to
what the chip delivers.

    python -m paper_1810_09784_amd.ceilings          # writes ceilings_gfx950.json
"""
import json
import os
import subprocess
import sys

from .build import CEILINGS, PKG

OUT = os.path.join(PKG, "ceilings_gfx950.json")


def run(timeout: int = 120) -> dict:
    if not os.path.exists(CEILINGS):
        raise RuntimeError(f"{CEILINGS} is not built: run paper_1810_09784_amd.build.build() first")
    r = subprocess.run([CEILINGS], capture_output=True, text=True, timeout=timeout)
    rows = [json.loads(l) for l in r.stdout.splitlines() if l.startswith("{")]
    if r.returncode != 0 or any("error" in x for x in rows):
        raise RuntimeError(f"ceilings run failed ({r.returncode}): {r.stdout}\n{r.stderr}")
    out = {"device": rows[0], "tests": {x["test"]: x for x in rows[1:]}}
    return out


def load():
    """The stored measurement, or None."""
    if not os.path.exists(OUT):
        return None
    with open(OUT) as f:
        return json.load(f)


def main():
    res = run()
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)
    for name, t in res["tests"].items():
        print(name, {k: v for k, v in t.items() if k != "test"}, flush=True)


if __name__ == "__main__":
    sys.exit(main())
