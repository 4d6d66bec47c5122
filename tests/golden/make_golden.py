"""Writes tests/golden/synth_sha256.json: SHA-256 of the generator's bytes for
the single-image workloads and the first images of the batch workload.  The
generator holds none of the segmentation arithmetic; these hashes only guard
the inputs against accidental change.  Calls nothing but ``synth``."""
import hashlib
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
import synth  # noqa: E402


def digests():
    out = {}
    for name, wl in synth.WORKLOADS.items():
        out[name] = hashlib.sha256(synth.image_for(wl).tobytes()).hexdigest()
    for wl in synth.batch_workload()[:4]:
        out[wl.name] = hashlib.sha256(synth.image_for(wl).tobytes()).hexdigest()
    return out


if __name__ == "__main__":
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "synth_sha256.json")
    with open(path, "w") as f:
        json.dump(digests(), f, indent=1, sort_keys=True)
        f.write("\n")
    print("wrote", path)
