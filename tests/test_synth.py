"""The seeded generators are deterministic and follow their error model."""
import json
import os

import numpy as np

import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def test_golden_hashes():
    import importlib.util
    spec = importlib.util.spec_from_file_location("mk", os.path.join(HERE, "golden", "make_synth_hashes.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    want = json.load(open(os.path.join(HERE, "golden", "synth_sha256.json")))
    assert mk.hashes() == want


def test_ranges_regenerate_identically():
    a = synth.workload("swg150", n=3000)
    b = synth.workload("swg150", start=1500, n=700)
    for i in range(b.n):
        assert np.array_equal(a.pattern(1500 + i), b.pattern(i))
        assert np.array_equal(a.text(1500 + i), b.text(i))


def test_error_model_statistics():
    b = synth.workload("swg150", n=20000)
    assert (b.txt_len == 150).all()
    # insertions and deletions are equally likely: mean pattern length ~ 150
    assert abs(b.pat_len.mean() - 150) < 0.1
    # each error type has rate 4 % / 3 per base: length variance = 150 * 2 * 0.04 / 3
    assert abs(b.pat_len.var() - 150 * 2 * 0.04 / 3) < 0.6
    w = synth.workload("wfa_mixed", n=4000)
    assert w.txt_len.min() >= 100 and w.txt_len.max() <= 10_000


def test_pack_roundtrip():
    b = synth.workload("wfa_mixed", n=50)
    words, woff = synth.pack_2bit(b.txt, b.txt_off)
    assert np.array_equal(synth.unpack_2bit(words, woff, b.txt_len), b.txt)
    assert (np.diff(woff) == (b.txt_len + 31) // 32).all()
