"""Writes synth_sha256.json: SHA-256 of the float32 bytes of each seeded generator output.

Run from the repository root:  python tests/golden/make_synth_fingerprints.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import synth  # noqa: E402


def fingerprints():
    out = {}
    for s in (0, 1):
        out["cube_%d" % s] = synth.fingerprint(synth.cube(s))
        out["room_%d" % s] = synth.fingerprint(synth.room(s))
        out["lidar_%d" % s] = synth.fingerprint(synth.lidar(s))
    xyz, off, m = synth.batch(0)
    out["batch_0"] = synth.fingerprint(xyz)
    out["batch_0_offsets"] = [int(v) for v in off]
    return out


if __name__ == "__main__":
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "synth_sha256.json")
    with open(path, "w") as f:
        json.dump(fingerprints(), f, indent=1, sort_keys=True)
    print("wrote", path)
