"""Property-based pins (Hypothesis, CPU only).

For random small dictionaries and texts over tiny alphabets, the C oracle,
the compiled trie walked on the host (whole patterns and truncated with
verification) and the truncated candidates must all equal the definition
written out by Python slicing (tests/brute.py).
"""

import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle
from brute import brute_matches

glop = pytest.importorskip("paper_1704_02278_amd")

alphabet = st.sampled_from([b"a", b"ab", b"abc", b"\x00\xff"])


@st.composite
def cases(draw):
    alpha = draw(alphabet)
    letters = st.sampled_from(list(alpha))
    word = st.lists(letters, min_size=1, max_size=12).map(bytes)
    pats = draw(st.lists(word, min_size=1, max_size=8))
    text = draw(st.lists(letters, min_size=0, max_size=200).map(bytes))
    return pats, text


@settings(max_examples=300, deadline=None)
@given(cases())
def test_oracle_equals_definition(case):
    pats, text = case
    want, want_counts = brute_matches(text, pats)
    for bucketed in (False, True):
        off, ids, counts, total = oracle.match(np.frombuffer(text, dtype=np.uint8), pats, bucketed=bucketed,
                                               threads=3)
        assert list(zip(off.tolist(), ids.tolist())) == want and counts.tolist() == want_counts


@settings(max_examples=300, deadline=None)
@given(cases(), st.integers(min_value=1, max_value=10))
def test_trie_engines_equal_definition(case, L):
    pats, text = case
    want = brute_matches(text, pats)
    for opts in (dict(prefix_len=glop.GLOP_PREFIX_FULL), dict(), dict(prefix_len=L)):
        off, ids, counts, total = glop.Dict(pats, device=False, **opts).cpu_walk(text, threads=2)
        assert (list(zip(off.tolist(), ids.tolist())), counts.tolist()) == want, opts
    off, ids, counts, total = glop.Dict(pats, device=False, prefix_len=L, candidates=True).cpu_walk(text)
    assert (list(zip(off.tolist(), ids.tolist())), counts.tolist()) == brute_matches(text, [p[:L] for p in pats])
