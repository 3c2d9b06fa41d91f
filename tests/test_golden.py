"""The stored oracle digests are reproducible: the generator still draws the
same pairs and the oracle still gives the same disparities (checked on the
smallest entries, CPU only)."""
import hashlib
import json
import os

import oracle
from paper_1610_04121_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_hashes.json")


def test_digests_reproduce_for_small_entries():
    doc = json.load(open(GOLDEN))
    assert (doc["P1"], doc["P2"]) == (synth.P1_DEFAULT, synth.P2_DEFAULT)
    small = sorted(doc["batch64"], key=lambda g: g["w"] * g["h"] * g["max_disp"] * g["n_paths"])[:2]
    for g in small:
        pr = synth.make_pair(g["w"], g["h"], g["max_disp"], g["scene"], seed=g["seed"])
        assert pr.sha_left == g["sha_left"] and pr.sha_right == g["sha_right"]
        out = oracle.sgm(pr.left, pr.right, g["max_disp"], doc["P1"], doc["P2"], g["n_paths"]).out
        assert hashlib.sha256(out.tobytes()).hexdigest() == g["out_sha256"]
    small = sorted(doc["batch64_median_lr"], key=lambda g: g["w"] * g["h"] * g["max_disp"] * g["n_paths"])[:1]
    for g in small:
        assert g["median"] and g["lr"]
        pr = synth.make_pair(g["w"], g["h"], g["max_disp"], g["scene"], seed=g["seed"])
        out = oracle.sgm(pr.left, pr.right, g["max_disp"], doc["P1"], doc["P2"], g["n_paths"], median=True,
                         lr=True).out
        assert hashlib.sha256(out.tobytes()).hexdigest() == g["out_sha256"]
        assert int((out == 0xFFFF).sum()) == g["invalid"]


def test_digest_entries_match_the_workload_definitions():
    doc = json.load(open(GOLDEN))
    items = synth.batch_items(64)
    for key in ("batch64", "batch64_median_lr"):
        assert [(i["w"], i["h"], i["max_disp"], i["n_paths"], i["seed"]) for i in items] == \
            [(g["w"], g["h"], g["max_disp"], g["n_paths"], g["seed"]) for g in doc[key]]
    kinds = synth.serve_kinds()
    assert [(k["w"], k["h"], k["max_disp"], k["seed"], k["scene"], k["scale_to_d"]) for k in kinds] == \
        [(g["w"], g["h"], g["max_disp"], g["seed"], g["scene"], g["scale_to_d"]) for g in doc["serve_kinds"]]
    # the smallest served kind reproduces on the CPU
    k = min(kinds, key=lambda k: k["w"] * k["h"] * k["max_disp"])
    g = next(g for g in doc["serve_kinds"] if (g["w"], g["h"], g["max_disp"]) == (k["w"], k["h"], k["max_disp"]))
    pr = synth.spec_pair(k)
    assert pr.sha_left == g["sha_left"]
