"""The seeded input generators (CPU only)."""

import collections

import numpy as np

import synth


def test_mt19937_64_reference_value():
    # The C++ standard fixes the 10000th output of mt19937_64 with its default
    # seed 5489 ([rand.predef]); the published reference code gives the same.
    assert int(synth.mt64_raw(5489, 10000)[-1]) == 9981545732273789042


def test_text_independent_of_thread_count():
    spec = synth.TextSpec(n_bytes=(3 << 20) + 12345, block_bytes=1 << 18)
    a = synth.gen_text(spec, 7, 99, threads=1)
    b = synth.gen_text(spec, 7, 99, threads=6)
    assert synth.sha256_bytes(a) == synth.sha256_bytes(b)
    c = synth.gen_text(spec, 8, 99, threads=6)
    assert synth.sha256_bytes(a) != synth.sha256_bytes(c)


def test_text_shape():
    spec = synth.TextSpec(n_bytes=2 << 20)
    t = synth.gen_text(spec, 11, 5)
    assert t.size == spec.n_bytes
    assert t[-1] == 0x0A
    allowed = np.zeros(256, dtype=bool)
    allowed[0x21:0x7F] = True
    allowed[0x20] = allowed[0x0A] = True
    assert allowed[t].all()
    nl = np.flatnonzero(t == 0x0A)
    starts = np.concatenate([[0], nl[:-1] + 1])
    content = nl - starts
    # all lines but a block's last are U{60..200}
    assert content.max() <= 200
    assert np.mean((content >= 60) & (content <= 200)) > 0.99
    assert abs(content.mean() - 130) < 3
    assert not np.any((t[:-1] == 0x20) & (t[1:] == 0x20))  # single spaces


def test_patterns_follow_spec():
    spec = synth.WORKLOADS["medium"].patterns
    pats = synth.gen_patterns(spec, 3, 17)
    assert len(pats) == 1000 and len(set(pats)) == 1000
    assert all(8 <= len(p) <= 64 for p in pats)
    assert all(0x20 <= b <= 0x7E for p in pats for b in p)
    exact = sum(any(q != p and q.startswith(p) for q in pats[:j]) for j, p in enumerate(pats))
    assert 0.03 * 1000 <= exact <= 0.08 * 1000
    assert pats == synth.gen_patterns(spec, 3, 17)


def test_zipf_lengths_short_heavy():
    spec = synth.WORKLOADS["large"].patterns
    pats = synth.gen_patterns(spec, 3, 19)
    lens = collections.Counter(len(p) for p in pats)
    assert min(lens) >= 4 and max(lens) <= 128
    assert lens[4] > lens[5] > lens[6] > lens[10]
    assert 0.22 < lens[4] / len(pats) < 0.32


def test_plants_are_inside_lines_and_slots():
    pats, text, plants = synth.make_workload("tiny")
    assert len(plants) == (1 << 20) // (4 << 10)
    every = synth.WORKLOADS["tiny"].text.plant_every
    for o, j in plants:
        p = pats[j]
        assert bytes(text[o:o + len(p)]) == p
        assert 0x0A not in p or True
        assert o // every == (o + len(p) - 1) // every
        assert 0x0A not in bytes(text[o:o + len(p)])


def test_draw_buffer_size_does_not_change_draws():
    a = synth.Draws(7, 11, chunk=3)
    b = synth.Draws(7, 11)
    assert [a.u32() for _ in range(1000)] == [b.u32() for _ in range(1000)]


def test_chunked_workload_shape():
    spec = synth.CHUNKED["batched"][1]
    sizes = synth.chunk_sizes(spec)
    assert len(sizes) == 4096 and min(sizes) >= 1 << 10 and max(sizes) <= 64 << 20
    med = sorted(sizes)[2048]
    assert 200 << 10 < med < 330 << 10  # lognormal median 256 KiB
    pats, text, offs, sz, plants = synth.make_chunks(count=40)
    assert sz == sizes[:40] and text.size == sum(sz)
    assert pats == synth.gen_patterns(synth.WORKLOADS["medium"].patterns, synth.BASE_SEED,
                                      synth.STREAM_PATTERNS + synth.WORKLOADS["medium"].index)
    for k in range(40):
        chunk = text[offs[k]:offs[k] + sz[k]]
        assert len(plants[k]) == sz[k] // spec.plant_every
        for o, j in plants[k]:
            assert chunk[o:o + len(pats[j])].tobytes() == pats[j]
        assert chunk[-1] == 0x0A  # every chunk ends a line


def test_pattern_set_hash_separates_boundaries():
    assert synth.sha256_patterns([b"ab", b"c"]) != synth.sha256_patterns([b"a", b"bc"])
    assert synth.sha256_patterns([b"ab", b"c"]) == synth.sha256_patterns([b"ab", b"c"])
    assert synth.sha256_patterns([]) == synth.sha256_bytes(b"")
