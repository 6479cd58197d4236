"""Brute-force definition of the match set, by Python slicing (tiny inputs only).

Independent of the C oracle: a different language and no shared code.  Used to
pin the oracle on small random inputs.
"""


def brute_matches(text: bytes, patterns: list[bytes]):
    pairs = []
    for i in range(len(text)):
        for j, p in enumerate(patterns):
            if text[i:i + len(p)] == p and i + len(p) <= len(text):
                pairs.append((i, j))
    counts = [0] * len(patterns)
    for _, j in pairs:
        counts[j] += 1
    return pairs, counts
