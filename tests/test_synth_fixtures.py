"""The synthetic inputs are byte-stable: every seeded generator (volumes, transfer functions,
lights, Gaussians, cameras, request logs) reproduces the SHA-256 digest stored in
tests/golden/synth_sha256.json (written by tests/golden/synth_fixtures.py).  A change of
numpy's or torch's generators or of a recipe shows up here before it shows up as a parity or
benchmark shift."""
import json
import os

from tests.golden.synth_fixtures import OUT, fixtures


def test_synthetic_fixtures_are_byte_stable():
    want = json.load(open(OUT))
    got = fixtures()
    assert sorted(got) == sorted(want)
    bad = [k for k in want if got[k] != want[k]]
    assert not bad, bad


def test_fixture_digests_repeat_within_a_process():
    assert fixtures() == fixtures()
