"""Writes the oracle's disparities, as SHA-256 digests, for the full-size
64-pair batch workload (without, and with median + left-right check on every
pair) and for each (size, disparity range) of the served request mix.  It
calls only the CPU oracle and the seeded generator; the GPU tests compare the
HIP path's outputs with these digests.

    python tests/golden/make_oracle_hashes.py     (a few minutes on 8 cores)
"""
import hashlib
import json
import os
import sys
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

P1, P2 = 7, 86


def _one(spec):
    import oracle
    from paper_1610_04121_amd import synth
    pair = synth.spec_pair(spec)
    out = oracle.sgm(pair.left, pair.right, spec["max_disp"], P1, P2, spec["n_paths"],
                     median=spec.get("median", False), lr=spec.get("lr", False)).out
    return dict(spec, sha_left=pair.sha_left, sha_right=pair.sha_right,
                out_sha256=hashlib.sha256(out.tobytes()).hexdigest(),
                invalid=int((out == 0xFFFF).sum()))


def main():
    import oracle
    from paper_1610_04121_amd import synth
    oracle.build()
    batch = synth.batch_items(64)
    batch_post = [dict(it, median=True, lr=True) for it in batch]
    serve = synth.serve_kinds()
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        b = pool.map(_one, batch, chunksize=1)
        bp = pool.map(_one, batch_post, chunksize=1)
        s = pool.map(_one, serve, chunksize=1)
    doc = {"P1": P1, "P2": P2, "census": "9x7 full", "batch64": b, "batch64_median_lr": bp, "serve_kinds": s}
    with open(os.path.join(HERE, "oracle_hashes.json"), "w") as f:
        json.dump(doc, f, indent=1)


if __name__ == "__main__":
    main()
