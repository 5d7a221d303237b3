"""The hash of Definition 1 pinned to published values, not to the oracle
itself: the SplitMix64 outputs of tests/golden/splitmix64.json (the
generator's published first outputs for seeds 0 and 1234567).  A mistyped
shift, multiplier or increment in the oracle's generator, its counter form
or its bucket and sign extraction changes these words."""
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.json")


def vectors():
    with open(GOLDEN) as f:
        doc = json.load(f)
    out = []
    for v in doc["vectors"]:
        words = [int(h, 16) for h in v["outputs_hex"]] if "outputs_hex" in v else [int(w) for w in v["outputs"]]
        out.append((int(v["seed"]), words))
    return out


@pytest.mark.parametrize("seed,words", vectors())
def test_stream_equals_published_outputs(orc, seed, words):
    got = orc.splitmix64_stream(seed, len(words))
    assert [int(w) for w in got] == words


@pytest.mark.parametrize("seed,words", vectors())
def test_row_hash_equals_published_outputs(orc, seed, words):
    # row i draws the (i+1)-th output: bucket from its high word, sign from bit 0
    for d in (2, 500, 20000, 2**31 - 1):
        bucket, sign = orc.hash_rows(seed, len(words), d)
        assert [int(b) for b in bucket] == [((w >> 32) * d) >> 32 for w in words]
        assert [int(s) for s in sign] == [-1 if (w & 1) else 1 for w in words]


def test_mix_function_equals_published_first_output(orc):
    # the first output of a generator seeded with 0 is mix(gamma), gamma the
    # generator's published increment
    assert orc.splitmix64_mix(0x9E3779B97F4A7C15) == vectors()[0][1][0]


def test_threaded_oracle_is_bitwise_the_single_thread_one(orc):
    # the sketch over bucket ranges and the loop's residual rows on several
    # threads: every entry keeps its sequential order, so the bits agree
    rng = np.random.default_rng(3)
    A = rng.standard_normal((6000, 37))
    xs = rng.standard_normal(37)
    b = A @ xs
    At1, bt1 = orc.sketch_dense(A, b, 700, 9)
    o1 = orc.mwrk(At1, bt1, xref=xs, tol=0.0, maxit=150, trace=True)
    with orc.threads(4) as t:
        assert t == 4
        At4, bt4 = orc.sketch_dense(A.astype(np.float32), b, 700, 9)
        At4d, bt4d = orc.sketch_dense(A, b, 700, 9)
        o4 = orc.mwrk(At4d, bt4d, xref=xs, tol=0.0, maxit=150, trace=True)
    At1f, _ = orc.sketch_dense(A.astype(np.float32), b, 700, 9)
    np.testing.assert_array_equal(At4d, At1)
    np.testing.assert_array_equal(bt4d, bt1)
    np.testing.assert_array_equal(At4, At1f)
    np.testing.assert_array_equal(o4.x, o1.x)
    np.testing.assert_array_equal(o4.idx, o1.idx)
