"""Writes input_hashes.json: SHA-256 fingerprints of the seeded inputs of the
small workloads.  Calls only the input generators (no GPU code, no oracle
arithmetic is needed for a fingerprint).  Run from the repository root:
    python tests/golden/make_input_hashes.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from paper_2502_04189_amd import workloads as W  # noqa: E402


def cases():
    yield "config0", W.config0()
    yield "random_48x36x20_wallz_tanh", W.random_case(7, 48, 36, 20, 0, 0, 1, stretch=1.8)
    for i, c in enumerate(W.config4(ndom=6)):
        yield f"config4_first6_{i}", c


if __name__ == "__main__":
    out = {name: W.fingerprint(c) for name, c in cases()}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "input_hashes.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print(json.dumps(out, indent=1))
