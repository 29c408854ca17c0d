"""The seeded input generators: determinism and the shape of the
primate-scale recipe (C generator), at a small scale."""
import numpy as np

import synth


def test_primate_is_deterministic_and_packs_like_pack():
    a = synth.primate(3, 0.0005)
    b = synth.primate(3, 0.0005, threads=1)
    assert len(a) == 8 and all(np.array_equal(x, y) for x, y in zip(a, b))
    for (pk, m, runs), codes in zip(synth.primate(3, 0.0005, packed=True), a):
        p2, r2 = synth.pack(codes)
        assert m == codes.size and np.array_equal(pk, p2) and np.array_equal(runs, r2)


def test_primate_shape():
    scale = 0.002
    gs = synth.primate(5, scale)
    n = int(3e9 * scale)
    for g, c in enumerate(gs):
        d = 0.005 + g * 0.035 / 7
        # indels change the length by a small fraction
        assert abs(c.size - n) < n * d
        assert c.max() == 4 and (c == 4).sum() >= 1000  # at least one N run
    # related genomes share most k-mers; the most diverged pair shares fewer
    def kmers(c, k=25):
        ok = c < 4
        v = np.zeros(c.size - k + 1, np.uint64)
        bad = np.zeros(c.size - k + 1, bool)
        for t in range(k):
            v = (v << np.uint64(2)) | c[t:t + v.size].astype(np.uint64) & np.uint64(3)
            bad |= ~ok[t:t + v.size]
        return set(v[~bad][:200000].tolist())
    k0, k1, k7 = kmers(gs[0]), kmers(gs[1]), kmers(gs[7])
    j01 = len(k0 & k1) / len(k0)
    j07 = len(k0 & k7) / len(k0)
    assert 0.15 < j07 < j01 < 0.95  # about (1 - d0 - d7)^25 for the pair (0, 7)


def test_primate_scale_and_seed_change_the_input():
    a = synth.primate(0, 0.0005)
    b = synth.primate(1, 0.0005)
    assert not np.array_equal(a[0][:10000], b[0][:10000])
