"""Pins of the oracle's random maps (CountSketch h and D, Section 1.3; modified
hash h~, Remark 2 / Proposition 4) against published values, closed forms and
statistics."""
import os

import numpy as np
import pytest

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_state0.txt")


def _golden():
    out = []
    for line in open(GOLD):
        line = line.strip()
        if line and not line.startswith("#"):
            out.append(int(line, 16))
    return out


def test_splitmix64_published_vectors():
    # seed 0, tag 0: key = mix64(0 ^ mix64(0)) = mix64(0) = 0, so the stream
    # is the published generator started at state 0.
    assert oracle.mix64(0) == 0
    assert oracle.lib().orc_stream_key(0, 0) == 0
    z = oracle.stream(0, 0, 3)
    assert [int(v) for v in z] == _golden()


def test_bucket_power_of_two_is_top_bits():
    # For L = 2^s the multiply-shift range map reduces to the top s bits of z.
    z = oracle.stream(7, 3, 4096)
    for s in (1, 4, 9, 16):
        b, _ = oracle.hash_maps(7, 3, 4096, 1 << s)
        assert np.array_equal(b.astype(np.uint64), z >> np.uint64(64 - s))


def test_sign_is_low_bit():
    z = oracle.stream(11, 0, 5000)
    _, s = oracle.hash_maps(11, 0, 5000, 37)
    assert np.array_equal(s, np.where((z & np.uint64(1)) == 0, 1, -1).astype(np.int8))


@pytest.mark.parametrize("L", [30, 128, 480, 4096])
def test_bucket_uniform_and_signs_balanced(L):
    m = 400_000
    b, s = oracle.hash_maps(0, 0, m, L)
    assert b.min() >= 0 and b.max() < L
    cnt = np.bincount(b, minlength=L)
    e = m / L
    chi2 = float(np.sum((cnt - e) ** 2 / e))
    # chi^2 with L-1 dof: mean L-1, sd sqrt(2(L-1)); allow 6 sd
    assert abs(chi2 - (L - 1)) < 6 * np.sqrt(2 * (L - 1))
    # +-1 with probability 1/2: |sum| within 6 sd
    assert abs(int(s.astype(np.int64).sum())) < 6 * np.sqrt(m)


def test_tags_give_independent_streams():
    m = 200_000
    _, s0 = oracle.hash_maps(5, 0, m, 64)
    _, s1 = oracle.hash_maps(5, 1, m, 64)
    _, s2 = oracle.hash_maps(6, 0, m, 64)
    for a, b in ((s0, s1), (s0, s2), (s1, s2)):
        c = float(np.mean(a.astype(np.float64) * b))
        assert abs(c) < 6 / np.sqrt(m)


def test_fullrank_hash_every_bucket_hit():
    # Remark 2: h~ = f o pi puts at least one row in every bucket.
    for seed in range(5):
        m, L = 1000, 333
        pi, x = synth.fullrank_perm(m, L, seed)
        b = oracle.fullrank_buckets(pi, x, L)
        assert b.min() >= 0 and b.max() < L
        assert np.all(np.bincount(b, minlength=L) >= 1)


def test_fullrank_collision_probability():
    # Proposition 4: P(h~(i) = h~(i')) = 1/L - (L-1)/(I(I-1)) for i != i'.
    m, L = 12, 5
    trials = 60_000
    hits = 0
    g = np.random.default_rng(3)
    for t in range(trials):
        pi = g.permutation(m).astype(np.int64)
        x = g.integers(0, L, size=m, dtype=np.int32)
        b = oracle.fullrank_buckets(pi, x, L)
        hits += int(b[0] == b[1])
    p_hat = hits / trials
    p = 1.0 / L - (L - 1) / (m * (m - 1))
    sd = np.sqrt(p * (1 - p) / trials)
    assert abs(p_hat - p) < 5 * sd
    # and the plain-hash probability 1/L is rejected at this size
    assert abs(p_hat - 1.0 / L) > 3 * sd

